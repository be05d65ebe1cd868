// Edge-tile shape of the BF16 MFMA chains: set, query, and a tuner that
// times afm_energy_forces on the caller's workload with every built shape
// and keeps the fastest (results are bitwise the same with every shape: an
// edge's MLP does not depend on which edges share its tile).
#include <hip/hip_runtime.h>

#include <string>

#include "internal.h"
#include "tune_cache.h"

namespace afm {

static std::string tune_key(const afm_model* m, int64_t n_atoms, int64_t n_edges) {
  const ModelDims& d = m->dims;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, m->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  std::string k = arch + "/w" + std::to_string(d.w) + "/c" + std::to_string(d.c) + "/l" + std::to_string(d.lmax) +
                  "/L" + std::to_string(d.NL) + "/d" + std::to_string(d.depth) + "/tb";
  for (int q = 0; q < d.ntb; ++q) k += (q ? "-" : "") + std::to_string(d.tb[q]);
  k += "/nb" + std::to_string(d.nb) + (m->fast_adjoint ? "/bf16fast" : "/bf16");
  const long long deg = n_atoms > 0 ? (long long)((double)n_edges / (double)n_atoms + 0.5) : 0;
  k += "/deg" + std::to_string(deg);
  return k;
}

}  // namespace afm

using namespace afm;

extern "C" {

int afm_set_edge_tile(afm_model* m, int32_t edges) {
  if (!m) { set_error("null model"); return AFM_E_INVALID; }
  if (edges != 64 && edges != 128) { set_error("edge tile must be 64 or 128"); return AFM_E_INVALID; }
  m->edge_tile = edges;
  return AFM_OK;
}

int afm_get_edge_tile(const afm_model* m, int32_t* edges) {
  if (!m || !edges) { set_error("null argument"); return AFM_E_INVALID; }
  *edges = m->prec == AFM_BF16_MFMA ? m->edge_tile : 0;
  return AFM_OK;
}

int afm_tune_edge_tile(afm_model* m, const afm_system* sys, const afm_nlist* nl, const afm_workspace* ws,
                       const char* cache_path, int32_t* chosen, double* ms, int32_t* from_cache, void* stream) {
  if (!m || !sys || !nl || !ws || !chosen) { set_error("null argument"); return AFM_E_INVALID; }
  if (ms) ms[0] = ms[1] = 0.0;
  if (from_cache) *from_cache = 0;
  if (m->prec != AFM_BF16_MFMA) { *chosen = 0; return AFM_OK; }   // no MFMA chains to tune
  hipStream_t st = (hipStream_t)stream;
  int64_t n_edges = 0;
  AFM_HIP_CHECK(hipMemcpyAsync(&n_edges, nl->n_edges, sizeof n_edges, hipMemcpyDeviceToHost, st));
  AFM_HIP_CHECK(hipStreamSynchronize(st));
  const std::string key = tune_key(m, sys->n_atoms, n_edges);
  TuneEntry e;
  if (tune_cache_lookup(cache_path, key, &e)) {
    m->edge_tile = e.tile;
    *chosen = e.tile;
    if (ms) { ms[0] = e.ms_64; ms[1] = e.ms_128; }
    if (from_cache) *from_cache = 1;
    return AFM_OK;
  }
  // scratch outputs for the timed evaluations
  const int64_t N = sys->n_atoms, B = sys->n_struct;
  double* buf = nullptr;
  AFM_HIP_CHECK(hipMalloc(&buf, sizeof(double) * (size_t)(N + B + 3 * N + 9 * B + 4)));
  double *e_atom = buf, *e_struct = buf + N, *F = e_struct + B, *W = F + 3 * N;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  int rc = AFM_OK;
  const int tiles[2] = {64, 128};
  double t_ms[2] = {0.0, 0.0};
  const int keep = m->edge_tile;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
    set_error("hipEventCreate failed");
    rc = AFM_E_HIP;
  }
  for (int v = 0; v < 2 && !rc; ++v) {
    m->edge_tile = tiles[v];
    rc = afm_energy_forces(m, sys, nl, e_atom, e_struct, F, W, ws, stream);   // warm-up
    const int reps = 3;
    if (!rc && hipEventRecord(t0, st) != hipSuccess) rc = AFM_E_HIP;
    for (int r = 0; r < reps && !rc; ++r) rc = afm_energy_forces(m, sys, nl, e_atom, e_struct, F, W, ws, stream);
    if (!rc && hipEventRecord(t1, st) != hipSuccess) rc = AFM_E_HIP;
    float el = 0.0f;
    if (!rc && (hipEventSynchronize(t1) != hipSuccess || hipEventElapsedTime(&el, t0, t1) != hipSuccess)) {
      set_error("timing the edge-tile variants failed");
      rc = AFM_E_HIP;
    }
    t_ms[v] = el / reps;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(buf);
  if (rc) { m->edge_tile = keep; return rc; }
  const int best = t_ms[1] < t_ms[0] ? 128 : 64;
  m->edge_tile = best;
  *chosen = best;
  if (ms) { ms[0] = t_ms[0]; ms[1] = t_ms[1]; }
  if (cache_path) {
    e.tile = best;
    e.ms_64 = t_ms[0];
    e.ms_128 = t_ms[1];
    if (!tune_cache_store(cache_path, key, e)) {
      set_error(std::string("could not write the tuning cache ") + cache_path);
      return AFM_E_INVALID;
    }
  }
  return AFM_OK;
}

}  // extern "C"
