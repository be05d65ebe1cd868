// Cache of instantiated hipGraphs of the MD sequence (host code only; no HIP
// types, so the key and eviction logic also builds and is tested with a plain
// C++ compiler).
//
// A captured sequence bakes in every device pointer, size and scalar that
// its kernels were launched with.  A graph may therefore be replayed only
// for exactly the same arguments, and only while every buffer it reads is
// alive.  The key holds
//   - the model's creation id (never reused, unlike the model's address or
//     its device allocation, which an allocator may hand out again),
//   - the workspace pointer, size and chunk plan,
//   - every system, neighbour-list and MD-state pointer, and
//   - every baked scalar (time step, skin, rebuild interval, thermostat
//     parameters, step phase, step count, atom and structure counts) and
//     the stream.
// Graphs of a model are destroyed when the model is (evict_model), and all
// remaining ones at process exit.
#pragma once
#include <stdint.h>
#include <string.h>

#include <functional>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/afm.h"

namespace afm {

struct GraphKey {
  uint64_t model_uid = 0;
  std::vector<uint64_t> words;
  bool operator<(const GraphKey& o) const {
    if (model_uid != o.model_uid) return model_uid < o.model_uid;
    return words < o.words;
  }
  bool operator==(const GraphKey& o) const { return model_uid == o.model_uid && words == o.words; }
  void add(const void* p) { words.push_back((uint64_t)(uintptr_t)p); }
  void add(int64_t v) { words.push_back((uint64_t)v); }
  void add(double v) {
    uint64_t u;
    memcpy(&u, &v, 8);
    words.push_back(u);
  }
};

// Everything an MD sequence launch depends on.
struct MdGraphFields {
  uint64_t model_uid;
  const afm_workspace* ws;
  int64_t n_atoms, n_struct;
  const void *species, *cell, *pbc, *seg;
  int64_t nl_capacity;
  const void *row_ptr, *col, *shift, *rev, *n_edges, *status;
  const afm_md_state* st;
  int64_t phase;
  int32_t n_steps;
  const void* stream;
};

inline GraphKey md_graph_key(const MdGraphFields& f) {
  GraphKey k;
  k.model_uid = f.model_uid;
  k.add(f.ws->ptr);
  k.add(f.ws->bytes);
  k.add(f.ws->chunk_edges);
  k.add(f.ws->n_chunks);
  k.add(f.ws->max_row);
  k.add(f.ws->edge_capacity);
  k.add((int64_t)f.ws->precision);
  k.add((int64_t)f.ws->with_second_order);
  k.add(f.n_atoms);
  k.add(f.n_struct);
  k.add(f.species);
  k.add(f.cell);
  k.add(f.pbc);
  k.add(f.seg);
  k.add(f.nl_capacity);
  k.add(f.row_ptr);
  k.add(f.col);
  k.add(f.shift);
  k.add(f.rev);
  k.add(f.n_edges);
  k.add(f.status);
  const afm_md_state* s = f.st;
  k.add((const void*)s->pos);
  k.add((const void*)s->vel);
  k.add((const void*)s->forces);
  k.add((const void*)s->mass_by_species);
  k.add((const void*)s->energy_log);
  k.add((const void*)s->e_atom);
  k.add((const void*)s->e_struct);
  k.add(s->dt_fs);
  k.add(s->skin);
  k.add((int64_t)s->rebuild_every);
  const bool nvt = s->t_target_K > 0;
  k.add(nvt ? s->t_target_K : 0.0);
  k.add(nvt ? s->tau_fs : 0.0);
  k.add(nvt ? s->n_dof : (int64_t)0);
  k.add(nvt ? (const void*)s->nh : nullptr);
  k.add(nvt ? (const void*)s->thermostat_log : nullptr);
  k.add(f.phase);
  k.add((int64_t)f.n_steps);
  k.add(f.stream);
  return k;
}

// Thread-safe map key -> executable graph; `destroy` releases one executable.
template <class Exec>
class GraphCache {
 public:
  explicit GraphCache(std::function<void(Exec)> destroy) : destroy_(std::move(destroy)) {}
  ~GraphCache() { clear(); }
  bool find(const GraphKey& k, Exec* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = map_.find(k);
    if (it == map_.end()) return false;
    *out = it->second;
    return true;
  }
  // Stores e under k; an executable already stored under k is destroyed.
  void insert(const GraphKey& k, Exec e) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = map_.find(k);
    if (it != map_.end()) {
      destroy_(it->second);
      it->second = e;
    } else {
      map_.emplace(k, e);
    }
  }
  // Destroys every graph captured with the model of this id; returns the count.
  size_t evict_model(uint64_t uid) {
    std::lock_guard<std::mutex> lk(mu_);
    size_t n = 0;
    for (auto it = map_.begin(); it != map_.end();) {
      if (it->first.model_uid == uid) {
        destroy_(it->second);
        it = map_.erase(it);
        ++n;
      } else {
        ++it;
      }
    }
    return n;
  }
  void clear() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : map_) destroy_(kv.second);
    map_.clear();
  }
  size_t size() {
    std::lock_guard<std::mutex> lk(mu_);
    return map_.size();
  }

 private:
  std::function<void(Exec)> destroy_;
  std::mutex mu_;
  std::map<GraphKey, Exec> map_;
};

}  // namespace afm
