// Host-side check of the MD graph cache (paper_2502_06073_amd/csrc/graph_cache.h):
// every baked argument is part of the key, and evicting a model destroys
// exactly its graphs.  Built with a plain C++ compiler by test_graph_cache.py.
#include <stdio.h>
#include <stdlib.h>

#include <set>
#include <vector>

#include "graph_cache.h"

using afm::GraphKey;
using afm::MdGraphFields;

static int fails = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #c); \
      ++fails;                                                \
    }                                                         \
  } while (0)

int main() {
  static char buf[64][64];
  afm_workspace ws{};
  ws.ptr = buf[0];
  ws.bytes = 1 << 20;
  ws.chunk_edges = 5000;
  ws.n_chunks = 3;
  ws.max_row = 1024;
  ws.edge_capacity = 15000;
  afm_md_state st{};
  st.pos = (double*)buf[1]; st.vel = (double*)buf[2]; st.forces = (double*)buf[3];
  st.mass_by_species = (const double*)buf[4]; st.energy_log = (double*)buf[5];
  st.e_atom = (double*)buf[6]; st.e_struct = (double*)buf[7];
  st.dt_fs = 0.5; st.skin = 0.5; st.rebuild_every = 10;
  MdGraphFields f{};
  f.model_uid = 7; f.ws = &ws; f.n_atoms = 100; f.n_struct = 1;
  f.species = buf[8]; f.cell = buf[9]; f.pbc = buf[10]; f.seg = buf[11];
  f.nl_capacity = 15000; f.row_ptr = buf[12]; f.col = buf[13]; f.shift = buf[14]; f.rev = buf[15];
  f.n_edges = buf[16]; f.status = buf[17]; f.st = &st; f.phase = 1; f.n_steps = 1; f.stream = buf[18];
  const GraphKey base = afm::md_graph_key(f);
  CHECK(afm::md_graph_key(f) == base);

  // every field, changed alone, gives another key
  std::vector<GraphKey> keys;
  auto vary = [&](auto&& change) {
    MdGraphFields g = f;
    afm_workspace w2 = ws;
    afm_md_state s2 = st;
    g.ws = &w2;
    g.st = &s2;
    change(g, w2, s2);
    keys.push_back(afm::md_graph_key(g));
  };
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.model_uid = 8; });
  vary([](MdGraphFields&, afm_workspace& w, afm_md_state&) { w.ptr = buf[20]; });
  vary([](MdGraphFields&, afm_workspace& w, afm_md_state&) { w.bytes += 256; });
  vary([](MdGraphFields&, afm_workspace& w, afm_md_state&) { w.chunk_edges = 6000; });
  vary([](MdGraphFields&, afm_workspace& w, afm_md_state&) { w.n_chunks = 4; });
  vary([](MdGraphFields&, afm_workspace& w, afm_md_state&) { w.max_row = 2048; });
  vary([](MdGraphFields&, afm_workspace& w, afm_md_state&) { w.edge_capacity = 16000; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.n_atoms = 101; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.n_struct = 2; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.species = buf[21]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.cell = buf[22]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.pbc = buf[23]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.seg = buf[24]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.nl_capacity = 15001; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.row_ptr = buf[25]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.col = buf[26]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.shift = buf[27]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.rev = buf[28]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.n_edges = buf[29]; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.status = buf[30]; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.pos = (double*)buf[31]; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.vel = (double*)buf[32]; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.forces = (double*)buf[33]; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.mass_by_species = (const double*)buf[34]; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.energy_log = (double*)buf[35]; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.e_atom = (double*)buf[36]; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.e_struct = (double*)buf[37]; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.dt_fs = 0.25; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.skin = 0.4; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) { s.rebuild_every = 20; });
  vary([](MdGraphFields&, afm_workspace&, afm_md_state& s) {
    s.t_target_K = 300.0; s.tau_fs = 100.0; s.nh = (double*)buf[38];
  });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.phase = 2; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.n_steps = 2; });
  vary([](MdGraphFields& g, afm_workspace&, afm_md_state&) { g.stream = buf[39]; });
  std::set<GraphKey> all(keys.begin(), keys.end());
  all.insert(base);
  CHECK(all.size() == keys.size() + 1);
  // NVT fields do not matter in NVE
  {
    afm_md_state s2 = st;
    s2.tau_fs = 55.0;
    s2.nh = (double*)buf[40];
    MdGraphFields g = f;
    g.st = &s2;
    CHECK(afm::md_graph_key(g) == base);
  }

  // eviction destroys exactly the model's graphs
  std::multiset<int> destroyed;
  {
    afm::GraphCache<int> cache([&](int e) { destroyed.insert(e); });
    MdGraphFields g = f;
    for (int k = 0; k < 6; ++k) {
      g.model_uid = 100 + (k % 2);
      g.phase = k;
      cache.insert(afm::md_graph_key(g), k);
    }
    CHECK(cache.size() == 6);
    int e = -1;
    g.model_uid = 100; g.phase = 2;
    CHECK(cache.find(afm::md_graph_key(g), &e) && e == 2);
    CHECK(cache.evict_model(100) == 3);
    CHECK(destroyed == std::multiset<int>({0, 2, 4}));
    CHECK(!cache.find(afm::md_graph_key(g), &e));
    g.model_uid = 101; g.phase = 3;
    CHECK(cache.find(afm::md_graph_key(g), &e) && e == 3);
    CHECK(cache.evict_model(100) == 0);
    // replacing an entry destroys the old executable
    cache.insert(afm::md_graph_key(g), 33);
    CHECK(destroyed.count(3) == 1 && cache.size() == 3);
  }
  // the cache's destructor releases what is left
  CHECK(destroyed == std::multiset<int>({0, 2, 4, 3, 1, 5, 33}));
  if (fails) return 1;
  printf("graph cache: %zu keys distinct, eviction ok\n", keys.size() + 1);
  return 0;
}
