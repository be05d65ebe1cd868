// Host-side check of the edge-tile tuner's cache (paper_2502_06073_amd/csrc/
// tune_cache.h): entries survive a format/parse round trip, a store adds or
// replaces one entry and keeps the others, malformed lines are skipped, and
// a missing file is a miss.  Built with a plain C++ compiler by
// test_tune_cache.py; argv[1] is a scratch file path.
#include <stdio.h>

#include <string>

#include "tune_cache.h"

static int fails = 0;
#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #c); \
      ++fails;                                                      \
    }                                                               \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const char* path = argv[1];
  remove(path);
  afm::TuneEntry e;
  CHECK(!afm::tune_cache_lookup(path, "k", &e));
  CHECK(afm::tile_shape_index(64, 8) == 0 && afm::tile_shape_index(128, 16) == 1 &&
        afm::tile_shape_index(128, 8) == 2 && afm::tile_shape_index(64, 16) < 0);
  afm::TuneEntry a, b;
  a.edges = 64; a.waves = 8; a.ms[0] = 11.25; a.ms[1] = 12.5; a.ms[2] = 11.5;
  b.edges = 128; b.waves = 8; b.ms[0] = 9.5; b.ms[1] = 9.75; b.ms[2] = 8.75;
  const char* k1 = "gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg72";
  const char* k2 = "gfx950/w256/c64/l2/L3/d3/tb64-128-256/nb8/bf16/deg61";
  CHECK(afm::tune_cache_store(path, k1, a));
  CHECK(afm::tune_cache_store(path, k2, b));
  CHECK(afm::tune_cache_lookup(path, k1, &e));
  CHECK(e.edges == 64 && e.waves == 8 && e.ms[0] == 11.25 && e.ms[1] == 12.5 && e.ms[2] == 11.5);
  CHECK(afm::tune_cache_lookup(path, k2, &e));
  CHECK(e.edges == 128 && e.waves == 8 && e.ms[2] == 8.75);
  CHECK(!afm::tune_cache_lookup(path, "gfx950/w256/c64/l2/L3/d3/tb64-128-256/nb8/bf16/deg60", &e));
  // replace one entry, keep the other
  afm::TuneEntry c;
  c.edges = 128; c.waves = 16; c.ms[0] = 11.0; c.ms[1] = 10.0; c.ms[2] = 10.5;
  CHECK(afm::tune_cache_store(path, k1, c));
  CHECK(afm::tune_cache_lookup(path, k1, &e));
  CHECK(e.edges == 128 && e.waves == 16 && e.ms[1] == 10.0);
  CHECK(afm::tune_cache_lookup(path, k2, &e));
  CHECK(e.edges == 128 && e.waves == 8 && e.ms[0] == 9.5);
  // malformed lines and unknown shapes are skipped
  auto m = afm::tune_cache_parse(
      "{\n\"x\": {\"edges\": 96, \"waves\": 8, \"ms_64x8\": 1}\n\"y\": {\"ms_64x8\": 1}\ngarbage\n"
      "\"z\": {\"edges\": 64, \"waves\": 8, \"ms_64x8\": 2.5, \"ms_128x16\": 3, \"ms_128x8\": 4}\n}\n");
  CHECK(m.size() == 1 && m.count("z") == 1 && m["z"].ms[0] == 2.5 && m["z"].ms[2] == 4.0);
  // round trip of the text form
  auto m2 = afm::tune_cache_parse(afm::tune_cache_format(m));
  CHECK(m2.size() == 1 && m2["z"].edges == 64 && m2["z"].ms[1] == 3.0);
  remove(path);
  if (fails) return 1;
  printf("tune cache ok\n");
  return 0;
}
