// NVE molecular dynamics step (Methodology: MD with a 0.5 fs time step).
// Velocity Verlet in float64:
//   v += dt/2 F/m k_acc;  r += dt v;
//   [k % rebuild_every == 0: wrap periodic atoms by whole lattice shifts,
//    rebuild the edge list at r_cut + skin];
//   [skin > 0: keep only the edges with |delta| < r_cut];
//   F = F(r);  v += dt/2 F/m k_acc;  log (KE, PE)
// with k_acc = 9.648533212e-3 A fs^-2 per (eV A^-1 amu^-1).  An atom that
// moved more than skin/2 since the last rebuild sets AFM_FLAG_SKIN.  The
// kinetic energy is reduced in a fixed order (per-block partials, then one
// block), so trajectories are bitwise reproducible.  Optionally the n-step
// sequence is captured once into a hipGraph and replayed.
//
// NVT (the paper's canonical-ensemble runs): one Nose-Hoover thermostat over
// all atoms, symmetric Trotter splitting around the Verlet step.  Each
// thermostat half step is one single-block kernel that reduces the kinetic
// energy partials, advances (xi, eta) in the device array nh and leaves the
// velocity scale exp(-xi dt/2) there; the scaling itself is folded into the
// next per-atom kernel.
#include <hip/hip_runtime.h>
#include <math.h>

#include <cstdlib>
#include <mutex>

#include "device_util.h"
#include "graph_cache.h"
#include "internal.h"
#include "trace.h"

namespace afm {

constexpr double kAcc = 9.648533212e-3;
constexpr double kKB = 8.617333262e-5;  // eV / K
constexpr int kMdBlock = 256;
// nh[]: thermostat state carried across steps and calls
constexpr int kNhXi = 0, kNhEta = 1, kNhScale = 2, kNhKe = 3;

// v = scale v + dt/2 F/m; r += dt v  (scale = nh[kNhScale] in NVT, else 1)
__global__ void k_md_kick_drift(double* __restrict__ pos, double* __restrict__ vel,
                                const double* __restrict__ F, const int32_t* __restrict__ species,
                                const double* __restrict__ mass, int S, int64_t N, double dt,
                                const double* __restrict__ ref, double half_skin2, int32_t* status,
                                const double* __restrict__ nh) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double inv_m = kAcc / mass[min(max(species[i], 0), S - 1)];
  const double sc = nh ? nh[kNhScale] : 1.0;
  double d2 = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double v = sc * vel[3 * i + q] + 0.5 * dt * F[3 * i + q] * inv_m;
    vel[3 * i + q] = v;
    const double r = pos[3 * i + q] + dt * v;
    pos[3 * i + q] = r;
    const double dd = r - ref[3 * i + q];
    d2 += dd * dd;
  }
  if (d2 > half_skin2) atomicOr(status, AFM_FLAG_SKIN);
}

__global__ void __launch_bounds__(kMdBlock) k_md_kick(double* __restrict__ vel, const double* __restrict__ F,
                                                       const int32_t* __restrict__ species,
                                                       const double* __restrict__ mass, int S, int64_t N, double dt,
                                                       double* __restrict__ ke_part) {
  __shared__ double part[kMdBlock];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double ke = 0.0;
  if (i < N) {
    const double m = mass[min(max(species[i], 0), S - 1)];
    const double inv_m = kAcc / m;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double v = vel[3 * i + q] + 0.5 * dt * F[3 * i + q] * inv_m;
      vel[3 * i + q] = v;
      ke += 0.5 * m * v * v / kAcc;
    }
  }
  part[threadIdx.x] = ke;
  __syncthreads();
  for (int off = kMdBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) ke_part[blockIdx.x] = part[0];
}

// per-block kinetic energy partials of the current velocities
__global__ void __launch_bounds__(kMdBlock) k_md_ke(const double* __restrict__ vel,
                                                     const int32_t* __restrict__ species,
                                                     const double* __restrict__ mass, int S, int64_t N,
                                                     double* __restrict__ ke_part) {
  __shared__ double part[kMdBlock];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double ke = 0.0;
  if (i < N) {
    const double m = mass[min(max(species[i], 0), S - 1)];
#pragma unroll
    for (int q = 0; q < 3; ++q) ke += 0.5 * m * vel[3 * i + q] * vel[3 * i + q] / kAcc;
  }
  part[threadIdx.x] = ke;
  __syncthreads();
  for (int off = kMdBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) ke_part[blockIdx.x] = part[0];
}

// One Nose-Hoover half step (time dt/2) from the kinetic energy partials:
// xi += dt/4 G(KE); s = exp(-xi dt/2); KE *= s^2; eta += xi dt/2;
// xi += dt/4 G(KE), G = (2 KE - gkT)/Q.  Leaves s and the scaled KE in nh;
// with tlog, writes Q xi^2/2 + gkT eta there.
__global__ void __launch_bounds__(256) k_nh_half(const double* __restrict__ ke_part, int64_t nb, double dt,
                                                  double Q, double gkT, double* __restrict__ nh,
                                                  double* __restrict__ tlog) {
  __shared__ double pa[256];
  double a = 0.0;
  for (int64_t k = threadIdx.x; k < nb; k += 256) a += ke_part[k];
  pa[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) pa[threadIdx.x] += pa[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double ke = pa[0], xi = nh[kNhXi], eta = nh[kNhEta];
    xi += 0.25 * dt * (2.0 * ke - gkT) / Q;
    const double s = exp(-0.5 * dt * xi);
    ke *= s * s;
    eta += 0.5 * dt * xi;
    xi += 0.25 * dt * (2.0 * ke - gkT) / Q;
    nh[kNhXi] = xi;
    nh[kNhEta] = eta;
    nh[kNhScale] = s;
    nh[kNhKe] = ke;
    if (tlog) *tlog = 0.5 * Q * xi * xi + gkT * eta;
  }
}

__global__ void k_md_scale(double* __restrict__ vel, int64_t n, const double* __restrict__ nh) {
  const double s = nh[kNhScale];
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    vel[q] *= s;
}

// (KE, PE) of the step; in NVT the KE after the thermostat scaling (nh)
__global__ void __launch_bounds__(256) k_md_log(const double* __restrict__ ke_part, int64_t nb,
                                                 const double* __restrict__ e_struct, int64_t B,
                                                 double* __restrict__ log2, const double* __restrict__ nh) {
  __shared__ double pa[256], pb[256];
  double a = 0.0, b = 0.0;
  for (int64_t k = threadIdx.x; k < nb; k += 256) a += ke_part[k];
  for (int64_t k = threadIdx.x; k < B; k += 256) b += e_struct[k];
  pa[threadIdx.x] = a;
  pb[threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      pa[threadIdx.x] += pa[threadIdx.x + off];
      pb[threadIdx.x] += pb[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    log2[0] = nh ? nh[kNhKe] : pa[0];
    log2[1] = pb[0];
  }
}

// r' = r - ((n0 a + n1 b) + n2 c), n = floor(frac(r)), only where n != 0
__global__ void k_md_wrap(double* __restrict__ pos, const double* __restrict__ cell,
                          const uint8_t* __restrict__ pbc, const int64_t* __restrict__ seg, int64_t B, int64_t N) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t lo = 0, hi = B;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (seg[mid] <= i) lo = mid; else hi = mid;
  }
  if (!pbc[lo]) return;
  const double* h = cell + 9 * lo;
  const double a[3] = {h[0], h[1], h[2]}, b[3] = {h[3], h[4], h[5]}, c[3] = {h[6], h[7], h[8]};
  const double bxc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
  const double cxa[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
  const double axb[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  const double det = a[0] * bxc[0] + a[1] * bxc[1] + a[2] * bxc[2];
  if (!(fabs(det) > 1e-12)) return;
  const double r[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  double n[3];
  n[0] = floor((r[0] * bxc[0] + r[1] * bxc[1] + r[2] * bxc[2]) / det);
  n[1] = floor((r[0] * cxa[0] + r[1] * cxa[1] + r[2] * cxa[2]) / det);
  n[2] = floor((r[0] * axb[0] + r[1] * axb[1] + r[2] * axb[2]) / det);
  if (n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0) return;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double s = __dadd_rn(__dadd_rn(__dmul_rn(n[0], h[q]), __dmul_rn(n[1], h[3 + q])), __dmul_rn(n[2], h[6 + q]));
    pos[3 * i + q] = __dsub_rn(r[q], s);
  }
}

__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    b[q] = a[q];
}

int api_energy_forces_dev(const afm_model* m, const SysDev& s, const NlDev& n, double* e_atom, double* e_struct,
                          double* forces, double* virial, const afm_workspace* ws, const WsLayout& L,
                          hipStream_t st);

static int md_sequence(const afm_model* m, const SysDev& s, const NlDev& n, const afm_md_state* state,
                       int32_t n_steps, const afm_workspace* ws, const WsLayout& L, hipStream_t st) {
  const int64_t N = s.N;
  const unsigned gb = grid_for(N, kMdBlock);
  double* ref = ws_ptr<double>(ws, L.md_ref);
  double* ke_part = ws_ptr<double>(ws, L.md_ke);
  const double r_list = m->dims.r_cut + state->skin;
  const double hs2 = 0.25 * state->skin * state->skin;
  const bool nvt = state->t_target_K > 0;
  double* nh = nvt ? state->nh : nullptr;
  const double gkT = (state->n_dof > 0 ? (double)state->n_dof : 3.0 * (double)N) * kKB * state->t_target_K;
  const double Q = gkT * state->tau_fs * state->tau_fs;
  if (state->step == 0) {
    hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(3 * N, 256, 4096)), dim3(256), 0, st, (const double*)state->pos,
                       ref, 3 * N);
  }
  for (int32_t t = 0; t < n_steps; ++t) {
    const int64_t k = state->step + t + 1;
    if (nvt) {
      hipLaunchKernelGGL(k_md_ke, dim3(gb), dim3(kMdBlock), 0, st, (const double*)state->vel, s.species,
                         state->mass_by_species, m->dims.S, N, ke_part);
      hipLaunchKernelGGL(k_nh_half, dim3(1), dim3(256), 0, st, (const double*)ke_part, (int64_t)gb, state->dt_fs, Q,
                         gkT, nh, (double*)nullptr);
    }
    hipLaunchKernelGGL(k_md_kick_drift, dim3(gb), dim3(kMdBlock), 0, st, state->pos, state->vel,
                       (const double*)state->forces, s.species, state->mass_by_species, m->dims.S, N, state->dt_fs,
                       (const double*)ref, hs2, n.status, (const double*)nh);
    AFM_LAUNCH_CHECK();
    if (state->rebuild_every > 0 && k % state->rebuild_every == 0) {
      hipLaunchKernelGGL(k_md_wrap, dim3(gb), dim3(256), 0, st, state->pos, s.cell, s.pbc, s.seg, s.B, N);
      int rc = launch_build_neighbors(s, r_list, n, ws, L, kMaxSpecies * 1024, st);
      if (rc) return rc;
      hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(3 * N, 256, 4096)), dim3(256), 0, st,
                         (const double*)state->pos, ref, 3 * N);
    }
    // with a skin, the edges beyond r_cut (exactly zero contributions) are
    // dropped before the per-edge pipeline
    NlDev nc = n;
    if (state->skin > 0) {
      int rc = launch_compact_to_cutoff(s, n, (float)m->dims.r_cut, ws, L, &nc, st);
      if (rc) return rc;
    }
    int rc = api_energy_forces_dev(m, s, nc, state->e_atom, state->e_struct, state->forces, nullptr, ws, L, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_md_kick, dim3(gb), dim3(kMdBlock), 0, st, state->vel, (const double*)state->forces,
                       s.species, state->mass_by_species, m->dims.S, N, state->dt_fs, ke_part);
    if (nvt) {
      hipLaunchKernelGGL(k_nh_half, dim3(1), dim3(256), 0, st, (const double*)ke_part, (int64_t)gb, state->dt_fs, Q,
                         gkT, nh, state->thermostat_log ? state->thermostat_log + t : (double*)nullptr);
      hipLaunchKernelGGL(k_md_scale, dim3(grid_for(3 * N, 256, 4096)), dim3(256), 0, st, state->vel, 3 * N,
                         (const double*)nh);
    }
    hipLaunchKernelGGL(k_md_log, dim3(1), dim3(256), 0, st, (const double*)ke_part, (int64_t)gb,
                       (const double*)state->e_struct, s.B, state->energy_log + 2 * (int64_t)t, (const double*)nh);
    AFM_LAUNCH_CHECK();
  }
  return AFM_OK;
}

// Instantiated graphs of MD sequences (graph_cache.h), created on first use
// (after HIP is initialised) together with an exit handler that destroys
// the graphs still cached; afm_model_destroy evicts the model's graphs.
static GraphCache<hipGraphExec_t>* g_cache = nullptr;
static std::once_flag g_cache_once;

static GraphCache<hipGraphExec_t>& graph_cache() {
  std::call_once(g_cache_once, [] {
    g_cache = new GraphCache<hipGraphExec_t>([](hipGraphExec_t e) { (void)hipGraphExecDestroy(e); });
    std::atexit([] {
      if (g_cache) g_cache->clear();
    });
  });
  return *g_cache;
}

void md_evict_model(uint64_t model_uid) {
  if (g_cache) g_cache->evict_model(model_uid);
}

int64_t md_cached_graphs() { return g_cache ? (int64_t)g_cache->size() : 0; }

int md_step(const afm_model* m, const SysDev& s, const NlDev& n, afm_md_state* state, int32_t n_steps,
            const afm_workspace* ws, const WsLayout& L, hipStream_t st) {
  TraceScope tr(st, "md_step");
  if (!state->use_graph || trace_on()) {
    int rc = md_sequence(m, s, n, state, n_steps, ws, L, st);
    if (!rc) state->step += n_steps;
    return rc;
  }
  if (state->step == 0 || !st) {
    // the reference capture at step 0 and the null stream are not captured
    int rc = md_sequence(m, s, n, state, n_steps, ws, L, st);
    if (!rc) state->step += n_steps;
    return rc;
  }
  const int64_t phase = state->rebuild_every > 0 ? state->step % state->rebuild_every : 0;
  MdGraphFields f{};
  f.model_uid = m->uid;
  f.ws = ws;
  f.n_atoms = s.N;
  f.n_struct = s.B;
  f.species = s.species;
  f.cell = s.cell;
  f.pbc = s.pbc;
  f.seg = s.seg;
  f.nl_capacity = n.capacity;
  f.row_ptr = n.row_ptr;
  f.col = n.col;
  f.shift = n.shift;
  f.rev = n.rev;
  f.n_edges = n.n_edges;
  f.status = n.status;
  f.st = state;
  f.phase = phase;
  f.n_steps = n_steps;
  f.stream = st;
  const GraphKey key = md_graph_key(f);
  hipGraphExec_t exec = nullptr;
  if (!graph_cache().find(key, &exec)) {
    AFM_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = md_sequence(m, s, n, state, n_steps, ws, L, st);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) { set_error(std::string("capture: ") + hipGetErrorString(e)); return AFM_E_HIP; }
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { set_error(std::string("graph instantiate: ") + hipGetErrorString(e)); return AFM_E_HIP; }
    graph_cache().insert(key, exec);
  }
  AFM_HIP_CHECK(hipGraphLaunch(exec, st));
  state->step += n_steps;
  return AFM_OK;
}

}  // namespace afm

extern "C" int64_t afm_md_graph_count(void) { return afm::md_cached_graphs(); }
