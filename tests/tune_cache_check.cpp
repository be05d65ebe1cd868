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
  afm::TuneEntry a{64, 11.25, 12.5}, b{128, 9.5, 8.75};
  CHECK(afm::tune_cache_store(path, "gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg72", a));
  CHECK(afm::tune_cache_store(path, "gfx950/w256/c64/l2/L3/d3/tb64-128-256/nb8/bf16/deg61", b));
  CHECK(afm::tune_cache_lookup(path, "gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg72", &e));
  CHECK(e.tile == 64 && e.ms_64 == 11.25 && e.ms_128 == 12.5);
  CHECK(afm::tune_cache_lookup(path, "gfx950/w256/c64/l2/L3/d3/tb64-128-256/nb8/bf16/deg61", &e));
  CHECK(e.tile == 128 && e.ms_128 == 8.75);
  CHECK(!afm::tune_cache_lookup(path, "gfx950/w256/c64/l2/L3/d3/tb64-128-256/nb8/bf16/deg60", &e));
  // replace one entry, keep the other
  afm::TuneEntry c{128, 11.0, 10.0};
  CHECK(afm::tune_cache_store(path, "gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg72", c));
  CHECK(afm::tune_cache_lookup(path, "gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg72", &e));
  CHECK(e.tile == 128 && e.ms_128 == 10.0);
  CHECK(afm::tune_cache_lookup(path, "gfx950/w256/c64/l2/L3/d3/tb64-128-256/nb8/bf16/deg61", &e));
  CHECK(e.tile == 128 && e.ms_64 == 9.5);
  // malformed lines and bad tiles are skipped
  auto m = afm::tune_cache_parse("{\n\"x\": {\"tile\": 96, \"ms_64\": 1}\n\"y\": {\"ms_64\": 1}\ngarbage\n"
                                 "\"z\": {\"tile\": 64, \"ms_64\": 2.5, \"ms_128\": 3}\n}\n");
  CHECK(m.size() == 1 && m.count("z") == 1 && m["z"].ms_64 == 2.5);
  // round trip of the text form
  auto m2 = afm::tune_cache_parse(afm::tune_cache_format(m));
  CHECK(m2.size() == 1 && m2["z"].tile == 64 && m2["z"].ms_128 == 3.0);
  remove(path);
  if (fails) return 1;
  printf("tune cache ok\n");
  return 0;
}
