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

int afm_set_edge_tile(afm_model* m, int32_t edges, int32_t waves) {
  if (!m) { set_error("null model"); return AFM_E_INVALID; }
  if (tile_shape_index(edges, waves) < 0) {
    set_error("edge-tile shape must be 64x8, 128x16 or 128x8 (edges x wavefronts)");
    return AFM_E_INVALID;
  }
  if (m->prec == AFM_BF16_MFMA && m->dims.w > 256 && edges != 64) {
    set_error("latent widths above 256 are built for 64-edge tiles only");
    return AFM_E_UNSUPPORTED;
  }
  m->edge_tile = edges;
  m->tile_waves = waves;
  return AFM_OK;
}

int afm_set_fused_last(afm_model* m, int32_t on, int32_t* active) {
  if (!m) { set_error("null model"); return AFM_E_INVALID; }
  m->fuse_last = on != 0;
  if (active) *active = (m->fuse_last && mfma_fused_last_available(m)) ? 1 : 0;
  return AFM_OK;
}

int afm_get_edge_tile(const afm_model* m, int32_t* edges, int32_t* waves) {
  if (!m || !edges || !waves) { set_error("null argument"); return AFM_E_INVALID; }
  const bool mfma = m->prec == AFM_BF16_MFMA;
  *edges = mfma ? m->edge_tile : 0;
  *waves = mfma ? m->tile_waves : 0;
  return AFM_OK;
}

int afm_tune_edge_tile(afm_model* m, const afm_system* sys, const afm_nlist* nl, const afm_workspace* ws,
                       const char* cache_path, int32_t* edges, int32_t* waves, double* ms, int32_t* from_cache,
                       void* stream) {
  if (!m || !sys || !nl || !ws || !edges || !waves) { set_error("null argument"); return AFM_E_INVALID; }
  if (ms)
    for (int q = 0; q < kTileShapes; ++q) ms[q] = 0.0;
  if (from_cache) *from_cache = 0;
  if (m->prec != AFM_BF16_MFMA) { *edges = *waves = 0; return AFM_OK; }   // no MFMA chains to tune
  hipStream_t st = (hipStream_t)stream;
  int64_t n_edges = 0;
  AFM_HIP_CHECK(hipMemcpyAsync(&n_edges, nl->n_edges, sizeof n_edges, hipMemcpyDeviceToHost, st));
  AFM_HIP_CHECK(hipStreamSynchronize(st));
  const std::string key = tune_key(m, sys->n_atoms, n_edges);
  TuneEntry e;
  if (tune_cache_lookup(cache_path, key, &e)) {
    m->edge_tile = *edges = e.edges;
    m->tile_waves = *waves = e.waves;
    if (ms)
      for (int q = 0; q < kTileShapes; ++q) ms[q] = e.ms[q];
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
  double t_ms[kTileShapes] = {};
  const int keep_e = m->edge_tile, keep_w = m->tile_waves;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
    set_error("hipEventCreate failed");
    rc = AFM_E_HIP;
  }
  for (int v = 0; v < kTileShapes && !rc; ++v) {
    t_ms[v] = -1.0;   // not built for this model
    if (m->dims.w > 256 && kTileEdges[v] != 64) continue;
    m->edge_tile = kTileEdges[v];
    m->tile_waves = kTileWaves[v];
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
  if (rc) { m->edge_tile = keep_e; m->tile_waves = keep_w; return rc; }
  int best = 0;
  for (int v = 1; v < kTileShapes; ++v)
    if (t_ms[v] >= 0.0 && t_ms[v] < t_ms[best]) best = v;
  m->edge_tile = *edges = kTileEdges[best];
  m->tile_waves = *waves = kTileWaves[best];
  if (ms)
    for (int q = 0; q < kTileShapes; ++q) ms[q] = t_ms[q];
  if (cache_path) {
    e.edges = kTileEdges[best];
    e.waves = kTileWaves[best];
    for (int q = 0; q < kTileShapes; ++q) e.ms[q] = t_ms[q];
    if (!tune_cache_store(cache_path, key, e)) {
      set_error(std::string("could not write the tuning cache ") + cache_path);
      return AFM_E_INVALID;
    }
  }
  return AFM_OK;
}

}  // extern "C"
