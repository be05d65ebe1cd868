// Per-edge kernels and the per-chunk forward / adjoint schedule.
//
// Forward (Methodology / Model Training; equations restated in the header of
// the library): geometry and basis -> two-body MLP -> for each layer L:
// environment embedding omega^L, environment sum + tensor products
// (tp_kernels.hip), latent MLP with residual -> edge energies -> per-atom
// and per-structure energies in float64.
// Adjoint: dE/dx from the linear edge-energy MLP, then every step in reverse
// (transposed-weight GEMMs, SiLU', tensor-product adjoint), ending in
// g_e = dE/d(delta_e) per edge; forces and virial are gathered per atom in
// float64 (F_i = sum_{row i} g_e - g_rev(e)), with no atomics.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device_util.h"
#include "edge_geom.h"
#include "gemm_f32.h"
#include "internal.h"
#include "trace.h"

namespace afm {

// BF16 MFMA chains (mfma_chain.hip)
int mfma_twobody_fwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                     const int32_t* species, const int32_t* col, hipStream_t st);
int mfma_latent_fwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer,
                    hipStream_t st);
int mfma_latent_bwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer,
                    const int32_t* species, const int64_t* seg, int64_t B, const double* grad_e_struct,
                    hipStream_t st);
int mfma_twobody_bwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                     const int32_t* species, hipStream_t st);
int mfma_latent_fb(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                   const int32_t* species, const int64_t* seg, int64_t B, const double* grad_e_struct, hipStream_t st);

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    p[q] = v;
}

int zero_async(void* p, int64_t bytes, hipStream_t st) {
  const int64_t n = bytes / 4;
  if (n <= 0) return AFM_OK;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, (uint32_t*)p, n, 0u);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

__device__ __forceinline__ double envelope_d(double x, int p) {
  if (x >= 1.0) return 0.0;
  const double xp = pow(x, (double)p);
  return 1.0 - 0.5 * (p + 1) * (p + 2) * xp + p * (p + 2) * xp * x - 0.5 * p * (p + 1) * xp * x * x;
}

__device__ __forceinline__ float envelope_f(float x, int p) {
  if (x >= 1.0f) return 0.0f;
  float xp = 1.0f;
  for (int q = 0; q < p; ++q) xp *= x;
  return 1.0f - 0.5f * (p + 1) * (p + 2) * xp + (float)(p * (p + 2)) * xp * x -
         0.5f * p * (p + 1) * xp * x * x;
}

// du/dx = -p(p+1)(p+2)/2 x^(p-1) (1 - x)^2
__device__ __forceinline__ float envelope_dx_f(float x, int p) {
  if (x >= 1.0f) return 0.0f;
  float xp = 1.0f;
  for (int q = 0; q < p - 1; ++q) xp *= x;
  return -0.5f * p * (p + 1) * (p + 2) * xp * (1.0f - x) * (1.0f - x);
}

// central atom of every edge of the chunk, geometry and basis inputs
__global__ void k_geometry(RowRange rr, const double* __restrict__ pos, const double* __restrict__ cell,
                           const uint8_t* __restrict__ pbc, const int64_t* __restrict__ seg, int64_t B,
                           const int32_t* __restrict__ col, const int8_t* __restrict__ shift, float r_cut,
                           int poly_p, int32_t* __restrict__ eidx, float* __restrict__ geo,
                           float* __restrict__ geo3) {
  const int64_t a0 = rr.chunk_rows[rr.chunk], a1 = rr.chunk_rows[rr.chunk + 1];
  const int64_t e0 = rr.row_ptr[a0], e1 = rr.row_ptr[a1];
  for (int64_t e = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < e1;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = a0, hi = a1;
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (rr.row_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    const int64_t i = lo, j = col[e];
    const int64_t sl = struct_of(seg, B, i);
    float dx, dy, dz;
    edge_vec_f32(pos, cell, pbc[sl] != 0, sl, i, j, shift + 3 * e, dx, dy, dz);
    const float r = edge_norm_f32(dx, dy, dz);
    const float inv = r > 0.0f ? 1.0f / r : 0.0f;
    const float u = envelope_f(r / r_cut, poly_p);
    const int64_t t = e - e0;
    float* g = geo + t * GEO_STRIDE;
    g[0] = dx; g[1] = dy; g[2] = dz; g[GEO_D] = r; g[GEO_U] = u;
    float Y[9];
    sh9(dx * inv, dy * inv, dz * inv, Y);
#pragma unroll
    for (int q = 0; q < 9; ++q) g[GEO_Y + q] = Y[q];
    g[14] = 0.0f; g[15] = 0.0f;
    if (geo3) {   // l_max = 3
      float Y3[7];
      sh_l3(dx * inv, dy * inv, dz * inv, Y3);
      float* g3 = geo3 + t * GEO3_STRIDE;
#pragma unroll
      for (int q = 0; q < 7; ++q) g3[q] = Y3[q];
      g3[7] = 0.0f;
    }
    eidx[t] = (int32_t)i;
  }
}

// first two-body layer: a[f] = W[f][Zi] + W[f][S + Zj] + sum_n W[f][2S + n] rho_n
__global__ void __launch_bounds__(256) k_twobody_first(RowRange rr, const int32_t* __restrict__ eidx,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ species,
                                                       const float* __restrict__ geo, const float* __restrict__ W,
                                                       int S, int nb, int F, float r_cut, float* __restrict__ pre,
                                                       int last, float* __restrict__ x0) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  __shared__ float rho[64][17];
  __shared__ int zz[64][2];
  const int64_t t0 = (int64_t)blockIdx.x * 64;
  if (t0 >= M) return;
  const int K = 2 * S + nb;
  if (threadIdx.x < 64) {
    const int64_t t = t0 + threadIdx.x;
    if (t < M) {
      const float r = geo[t * GEO_STRIDE + GEO_D], u = geo[t * GEO_STRIDE + GEO_U];
      const float c = sqrtf(2.0f / r_cut) / r;
      for (int q = 0; q < nb; ++q) rho[threadIdx.x][q] = c * sinf((q + 1) * 3.14159265358979323846f * r / r_cut) * u;
      rho[threadIdx.x][16] = u;
      // species outside [0, S) are clamped here and flagged by the energy kernel
      zz[threadIdx.x][0] = min(max(species[eidx[t]], 0), S - 1);
      zz[threadIdx.x][1] = min(max(species[col[e0 + t]], 0), S - 1);
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * F; idx += 256) {
    const int tl = idx / F, f = idx % F;
    const int64_t t = t0 + tl;
    if (t >= M) continue;
    const float* w = W + (int64_t)f * K;
    float a = w[zz[tl][0]] + w[S + zz[tl][1]];
    for (int q = 0; q < nb; ++q) a += w[2 * S + q] * rho[tl][q];
    pre[t * F + f] = a;
    if (last) x0[t * F + f] = rho[tl][16] * silu_f(a);
  }
}

// eps_e = w_eff . x (one wavefront per edge)
__global__ void __launch_bounds__(256) k_edge_energy(RowRange rr, const float* __restrict__ x, int w,
                                                     const float* __restrict__ w_eff, float* __restrict__ eps) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  const int lane = threadIdx.x & 63;
  for (int64_t t = blockIdx.x * 4 + (threadIdx.x >> 6); t < M; t += (int64_t)gridDim.x * 4) {
    float acc = 0.0f;
    for (int f = lane; f < w; f += 64) acc += w_eff[f] * x[t * w + f];
    acc = group_sum<64>(acc);
    if (lane == 0) eps[e0 + t] = acc;
  }
}

// Per-atom row reductions run on groups of kRowLanes consecutive lanes, one
// group per atom: the lanes of a group read consecutive edges of the row
// (coalesced), and a row of ~70 edges takes ~5 steps instead of ~70, so
// even a 10^4-atom system fills the chip.
constexpr int kRowLanes = 16;
constexpr int kRowBlock = 256;

// Sum over a lane group (butterfly: every lane of the group ends with the
// same bits, and the order is fixed, so the result repeats run to run)
__device__ __forceinline__ double row_group_sum(double v) {
#pragma unroll
  for (int o = kRowLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// E_i = sigma_Z energy_scale sum_{row i} eps_e + mu_Z (float64)
__global__ void __launch_bounds__(kRowBlock) k_atom_energy(const int64_t* __restrict__ row_ptr, int64_t N,
                                                           int64_t capacity, const float* __restrict__ eps,
                                                           const int32_t* __restrict__ species, int n_species,
                                                           const double* __restrict__ sc,
                                                           const double* __restrict__ sh, double escale,
                                                           double* __restrict__ e_atom, int32_t* status) {
  const int64_t i = (blockIdx.x * (int64_t)kRowBlock + threadIdx.x) / kRowLanes;
  const int sub = threadIdx.x % kRowLanes;
  if (i >= N) return;   // uniform over the lane group
  const int zi = species[i];
  if (row_ptr[N] > capacity || zi < 0 || zi >= n_species) {
    if (sub == 0) {
      if (zi < 0 || zi >= n_species) atomicOr(status, AFM_FLAG_SPECIES);
      e_atom[i] = __longlong_as_double(0x7ff8000000000000LL);
    }
    return;
  }
  double acc = 0.0;
  for (int64_t e = row_ptr[i] + sub; e < row_ptr[i + 1]; e += kRowLanes) acc += (double)eps[e];
  acc = row_group_sum(acc);
  if (sub == 0) e_atom[i] = sc[zi] * escale * acc + sh[zi];
}

// per-structure sums of per-atom values: strided per-thread sums, a
// butterfly per wavefront, then the wavefront partials in order (fixed
// order throughout)
constexpr int kSumBlock = 1024;
template <int W>
__global__ void __launch_bounds__(kSumBlock) k_struct_sum(const int64_t* __restrict__ seg,
                                                          const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double part[kSumBlock / 64][W];
  const int64_t s = blockIdx.x;
  const int64_t a = seg[s], b = seg[s + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[W];
#pragma unroll
  for (int q = 0; q < W; ++q) acc[q] = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += kSumBlock)
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] += v[i * W + q];
#pragma unroll
  for (int q = 0; q < W; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
    if (lane == 0) part[wave][q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x < W) {
    double t = 0.0;
    for (int w = 0; w < kSumBlock / 64; ++w) t += part[w][threadIdx.x];
    out[s * W + threadIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// backward elementwise pieces

// dE/dx^{NL}[t][f] = sigma_Z(i) escale gE_s w_eff[f]
__global__ void k_gx_init(RowRange rr, const int32_t* __restrict__ eidx, const int32_t* __restrict__ species,
                          const int64_t* __restrict__ seg, int64_t B, const double* __restrict__ ges,
                          const double* __restrict__ sc, int S, double escale, const float* __restrict__ w_eff,
                          int w, float* __restrict__ gx) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t n = (e1 - e0) * w;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / w;
    const int f = (int)(q % w);
    const int64_t i = eidx[t];
    double c = sc[min(max(species[i], 0), S - 1)] * escale;
    if (ges) {
      int64_t lo = 0, hi = B;
      while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (seg[mid] <= i) lo = mid; else hi = mid;
      }
      c *= ges[lo];
    }
    gx[q] = (float)c * w_eff[f];
  }
}

// Head of an MLP adjoint whose output is y = res*(x_prev) + u * silu(a):
//   ga = gy_coef * gx * u * silu'(a);  gu += sum_f gy_coef * gx * silu(a);
//   gx <- res_coef * gx  (the residual share, kept in place)
// one wavefront per edge.
__global__ void __launch_bounds__(256) k_mlp_head_bwd(RowRange rr, int w, const float* __restrict__ a,
                                                      const float* __restrict__ geo, float coef, float res_coef,
                                                      float* __restrict__ gx, float* __restrict__ ga,
                                                      float* __restrict__ gy) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  const int lane = threadIdx.x & 63;
  for (int64_t t = blockIdx.x * 4 + (threadIdx.x >> 6); t < M; t += (int64_t)gridDim.x * 4) {
    const float u = geo[t * GEO_STRIDE + GEO_U];
    float gu = 0.0f;
    for (int f = lane; f < w; f += 64) {
      const float g = coef * gx[t * w + f];
      const float av = a[t * w + f];
      ga[t * w + f] = g * u * dsilu_f(av);
      gu += g * silu_f(av);
      gx[t * w + f] = res_coef * gx[t * w + f];
    }
    gu = group_sum<64>(gu);
    if (lane == 0) gy[t * GEO_STRIDE + 9] += gu;
  }
}

// g_e = dE/d delta_e from dE/drho, dE/du and dE/dY
__global__ void k_geometry_bwd(RowRange rr, const float* __restrict__ geo, const float* __restrict__ grho,
                               const float* __restrict__ gy, const float* __restrict__ gy3, int nb, float r_cut,
                               int poly_p, float* __restrict__ g) {
  int64_t e0, e1;
  rr.get(e0, e1);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < e1 - e0;
       t += (int64_t)gridDim.x * blockDim.x) {
    const float* G = geo + t * GEO_STRIDE;
    const float r = G[GEO_D];
    const float dx = G[0], dy = G[1], dz = G[2];
    float out[3] = {0.0f, 0.0f, 0.0f};
    if (r > 0.0f) {
      const float inv = 1.0f / r;
      const float ux = dx * inv, uy = dy * inv, uz = dz * inv;
      const float x = r / r_cut;
      const float u = G[GEO_U];
      const float du = envelope_dx_f(x, poly_p) / r_cut;
      const float c = sqrtf(2.0f / r_cut);
      float gd = gy[t * GEO_STRIDE + 9] * du;
      for (int q = 0; q < nb; ++q) {
        const float k = (q + 1) * 3.14159265358979323846f / r_cut;
        const float sn = sinf(k * r), cs = cosf(k * r);
        const float B = c * sn * inv;
        const float dB = c * (k * cs * inv - sn * inv * inv);
        gd += grho[t * 16 + q] * (dB * u + B * du);
      }
      float gu3[3];
      sh9_grad(ux, uy, uz, gy + t * GEO_STRIDE, gu3);
      if (gy3) sh_l3_grad(ux, uy, uz, gy3 + t * GEO3_STRIDE, gu3);   // l_max = 3
      const float dot = gu3[0] * ux + gu3[1] * uy + gu3[2] * uz;
      out[0] = gd * ux + (gu3[0] - dot * ux) * inv;
      out[1] = gd * uy + (gu3[1] - dot * uy) * inv;
      out[2] = gd * uz + (gu3[2] - dot * uz) * inv;
    }
    float* o = g + (e0 + t) * 3;
    o[0] = out[0]; o[1] = out[1]; o[2] = out[2];
  }
}

// F_i = sum_{e in row i} (g_e - g_rev(e));  W_i = -sum_{e in row i} g_e delta_e^T
// (one lane group per atom)
__global__ void __launch_bounds__(kRowBlock) k_force_scatter(const double* __restrict__ pos, const double* __restrict__ cell,
                                const uint8_t* __restrict__ pbc, const int64_t* __restrict__ seg, int64_t B,
                                const int64_t* __restrict__ row_ptr, int64_t N, const int32_t* __restrict__ col,
                                const int8_t* __restrict__ shift, const int32_t* __restrict__ rev,
                                const float* __restrict__ g, int64_t capacity, double* __restrict__ forces,
                                double* __restrict__ wat) {
  const int64_t i = (blockIdx.x * (int64_t)kRowBlock + threadIdx.x) / kRowLanes;
  const int sub = threadIdx.x % kRowLanes;
  if (i >= N) return;   // uniform over the lane group
  if (row_ptr[N] > capacity) {
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    if (sub == 0) {
      if (forces) for (int q = 0; q < 3; ++q) forces[3 * i + q] = nan;
      if (wat) for (int q = 0; q < 9; ++q) wat[9 * i + q] = nan;
    }
    return;
  }
  int64_t sl = 0, sh = B;
  while (sh - sl > 1) {
    int64_t mid = (sl + sh) >> 1;
    if (seg[mid] <= i) sl = mid; else sh = mid;
  }
  const bool per = pbc[sl] != 0;
  const double* h = cell + 9 * sl;
  double F[3] = {0, 0, 0}, Wv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t e = row_ptr[i] + sub; e < row_ptr[i + 1]; e += kRowLanes) {
    const int64_t j = col[e], r = rev[e];
    float ge[3] = {g[3 * e], g[3 * e + 1], g[3 * e + 2]};
    double d[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
      if (per)
        s = __dadd_rn(__dadd_rn(__dmul_rn((double)shift[3 * e], h[q]), __dmul_rn((double)shift[3 * e + 1], h[3 + q])),
                      __dmul_rn((double)shift[3 * e + 2], h[6 + q]));
      d[q] = (double)(float)__dadd_rn(__dsub_rn(pos[3 * j + q], pos[3 * i + q]), s);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      F[q] += (double)ge[q] - (r >= 0 ? (double)g[3 * r + q] : 0.0);
#pragma unroll
      for (int p = 0; p < 3; ++p) Wv[q * 3 + p] -= (double)ge[q] * d[p];
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) F[q] = row_group_sum(F[q]);
  if (wat)
#pragma unroll
    for (int q = 0; q < 9; ++q) Wv[q] = row_group_sum(Wv[q]);
  if (sub != 0) return;
  if (forces)
    for (int q = 0; q < 3; ++q) forces[3 * i + q] = F[q];
  if (wat)
    for (int q = 0; q < 9; ++q) wat[9 * i + q] = Wv[q];
}

// ---------------------------------------------------------------------------
// loaders / epilogues for the FP32 GEMMs

struct LoadPlain {
  const float* x; int ld;
  __device__ float operator()(int m, int k) const { return x[(int64_t)m * ld + k]; }
};
struct LoadSilu {
  const float* a; int ld;
  __device__ float operator()(int m, int k) const { return silu_f(a[(int64_t)m * ld + k]); }
};
struct LoadCat {
  const float* x; int w; const float* s; int ls;
  __device__ float operator()(int m, int k) const {
    return k < w ? x[(int64_t)m * w + k] : s[(int64_t)m * ls + (k - w)];
  }
};
struct EpStore {
  float* y; int ld;
  __device__ void operator()(int m, int n, float v) const { y[(int64_t)m * ld + n] = v; }
};
struct EpAdd {
  float* y; int ld;
  __device__ void operator()(int m, int n, float v) const { y[(int64_t)m * ld + n] += v; }
};
// store pre-activation and y = u silu(a)  (two-body output)
struct EpTwobodyOut {
  float* pre; float* x; const float* geo; int ld;
  __device__ void operator()(int m, int n, float v) const {
    pre[(int64_t)m * ld + n] = v;
    x[(int64_t)m * ld + n] = geo[(int64_t)m * GEO_STRIDE + GEO_U] * silu_f(v);
  }
};
// store pre-activation and x_new = (x_prev + u silu(a)) / sqrt 2
struct EpLatentOut {
  float* pre; const float* xprev; float* xnew; const float* geo; int ld;
  __device__ void operator()(int m, int n, float v) const {
    pre[(int64_t)m * ld + n] = v;
    xnew[(int64_t)m * ld + n] =
        (xprev[(int64_t)m * ld + n] + geo[(int64_t)m * GEO_STRIDE + GEO_U] * silu_f(v)) * 0.70710678118654752f;
  }
};
// ga_prev = acc * silu'(a_prev)
struct EpDsilu {
  const float* a; float* ga; int ld;
  __device__ void operator()(int m, int n, float v) const {
    ga[(int64_t)m * ld + n] = v * dsilu_f(a[(int64_t)m * ld + n]);
  }
};
// split [x | s]-gradient: first w columns added to gx, rest stored to gs
struct EpSplit {
  float* gx; int w; float* gs; int ls;
  __device__ void operator()(int m, int n, float v) const {
    if (n < w) gx[(int64_t)m * w + n] += v; else gs[(int64_t)m * ls + (n - w)] = v;
  }
};

// ---------------------------------------------------------------------------
// schedule

static RowRange row_range(const NlDev& nl, const afm_workspace* ws, const WsLayout& L, int chunk) {
  RowRange rr;
  rr.chunk_rows = ws_ptr<int64_t>(ws, L.chunk_rows);
  rr.row_ptr = nl.row_ptr;
  rr.chunk = chunk;
  return rr;
}

static TPArgs tp_args(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer) {
  const ModelDims& d = m->dims;
  TPArgs a{};
  a.rr = rr;
  a.geo = ws_ptr<float>(ws, L.geo);
  a.omega = ws_ptr<float>(ws, L.omega[layer - 1]);
  a.omega1 = ws_ptr<float>(ws, L.omega[0]);
  for (int l = 0; l < d.NL; ++l) {
    a.gamma_l[l] = ws_ptr<float>(ws, L.gamma[l]);
    a.alpha_l[l] = l + 1 < d.NL ? m->W.alpha[l] : nullptr;
    a.gs_l[l] = ws_ptr<float>(ws, L.gs[l]);   // bf16 bits in the BF16 path
  }
  a.s = ws_ptr<float>(ws, L.s[layer - 1]);
  a.gamma = ws_ptr<float>(ws, L.gamma[layer - 1]);
  a.alpha = layer < d.NL ? m->W.alpha[layer - 1] : nullptr;
  a.inv_sqrt_nbar = (float)(1.0 / sqrt(d.nbar));
  a.gy = ws_ptr<float>(ws, L.gy);
  a.geo3 = d.lmax == 3 ? ws_ptr<float>(ws, L.geo3) : nullptr;
  a.gy3 = d.lmax == 3 ? ws_ptr<float>(ws, L.gy3) : nullptr;
  a.gomega = ws_ptr<float>(ws, L.gomega);
  return a;
}

static DenseArgs dense_args(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer) {
  DenseArgs a{};
  a.rr = rr;
  a.geo = ws_ptr<float>(ws, L.geo);
  a.omega = ws_ptr<float>(ws, L.omega[layer - 1]);
  a.omega1 = ws_ptr<float>(ws, L.omega[0]);
  a.s = ws_ptr<float>(ws, L.s[layer - 1]);
  a.gamma = ws_ptr<float>(ws, L.gamma[layer - 1]);
  a.vin = layer >= 2 ? ws_ptr<float>(ws, L.dense_v[layer - 2]) : nullptr;
  a.tbuf = ws_ptr<float>(ws, L.dense_t);
  a.dvbuf = ws_ptr<float>(ws, L.dense_dv);
  a.gs = ws_ptr<float>(ws, L.gs[layer - 1]);
  a.gomega = ws_ptr<float>(ws, L.gomega);
  a.gy = ws_ptr<float>(ws, L.gy);
  a.inv_sqrt_nbar = (float)(1.0 / sqrt(m->dims.nbar));
  return a;
}

// tensor products of one layer: the per-path kernels, or with dense mixing
// the stored-feature kernels and (below the last layer) the mixing GEMMs
static int tensor_products(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer,
                           bool bwd, int64_t n_atoms, hipStream_t st) {
  const ModelDims& d = m->dims;
  const bool bf16 = m->prec == AFM_BF16_MFMA;
  if (!(d.dense && d.NL > 1)) {
    TraceScope tr(st, bwd ? "tp_bwd" : "tp_fwd", layer);
    return launch_tp(d.lmax, d.NL, layer, d.c, bwd, bf16, tp_args(m, ws, L, rr, layer), n_atoms, st);
  }
  const DenseArgs a = dense_args(m, ws, L, rr, layer);
  int rc = AFM_OK;
  if (bwd && layer < d.NL) {   // dE/dT^L from dE/dV^L (left in dvbuf by layer L + 1)
    TraceScope tr(st, "mix_bwd", layer);
    rc = launch_dense_mix(m, layer, true, rr, L.cex, a.dvbuf, a.tbuf, st);
    if (rc) return rc;
  }
  {
    TraceScope tr(st, bwd ? "tp_bwd" : "tp_fwd", layer);
    rc = launch_dense_tp(d.lmax, d.NL, layer, d.c, bwd, bf16, a, n_atoms, st);
    if (rc) return rc;
  }
  if (!bwd && layer < d.NL) {
    TraceScope tr(st, "mix_fwd", layer);
    rc = launch_dense_mix(m, layer, false, rr, L.cex, ws_ptr<float>(ws, L.dense_v[layer - 1]), a.tbuf, st);
  }
  return rc;
}

int launch_geometry(const afm_model* m, const SysDev& s, const NlDev& nl, const afm_workspace* ws, const WsLayout& L,
                    RowRange rr, hipStream_t st) {
  hipLaunchKernelGGL(k_geometry, dim3(grid_for(L.cex, 256, 65536)), dim3(256), 0, st, rr, s.pos, s.cell, s.pbc,
                     s.seg, s.B, (const int32_t*)nl.col, (const int8_t*)nl.shift, (float)m->dims.r_cut, m->dims.p,
                     ws_ptr<int32_t>(ws, L.eidx), ws_ptr<float>(ws, L.geo),
                     m->dims.lmax == 3 ? ws_ptr<float>(ws, L.geo3) : nullptr);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

int run_forward_chunk(const afm_model* m, const SysDev& s, const NlDev& nl, const afm_workspace* ws,
                      const WsLayout& L, int chunk, hipStream_t st, bool fused_last) {
  const ModelDims& d = m->dims;
  const Plan& P = m->plan;
  RowRange rr = row_range(nl, ws, L, chunk);
  const int64_t E = L.cex;
  float* geo = ws_ptr<float>(ws, L.geo);
  int32_t* eidx = ws_ptr<int32_t>(ws, L.eidx);
  const int cw = (d.lmax + 1) * d.c;
  {
    TraceScope tr(st, "geometry");
    hipLaunchKernelGGL(k_geometry, dim3(grid_for(E, 256, 65536)), dim3(256), 0, st, rr, s.pos, s.cell, s.pbc,
                       s.seg, s.B, (const int32_t*)nl.col, (const int8_t*)nl.shift, (float)d.r_cut, d.p, eidx,
                       geo, d.lmax == 3 ? ws_ptr<float>(ws, L.geo3) : nullptr);
    AFM_LAUNCH_CHECK();
  }
  if (m->prec == AFM_BF16_MFMA) {
    TraceScope tr(st, "twobody_fwd");
    int rc = mfma_twobody_fwd(m, ws, L, rr, s.species, nl.col, st);
    if (rc) return rc;
  } else {
    TraceScope tr(st, "twobody_fwd");
    float* pre0 = ws_ptr<float>(ws, L.tb_pre[0]);
    hipLaunchKernelGGL(k_twobody_first, dim3(grid_for(E, 64)), dim3(256), 0, st, rr, (const int32_t*)eidx,
                       (const int32_t*)nl.col, s.species, (const float*)geo, m->W.tb[0], d.S, d.nb, d.tb[0],
                       (float)d.r_cut, pre0, d.ntb == 1 ? 1 : 0, ws_ptr<float>(ws, L.x[0]));
    AFM_LAUNCH_CHECK();
    for (int k = 1; k < d.ntb; ++k) {
      const float* ain = ws_ptr<float>(ws, L.tb_pre[k - 1]);
      float* pre = ws_ptr<float>(ws, L.tb_pre[k]);
      if (k == d.ntb - 1)
        sgemm<true>(st, rr, E, d.tb[k - 1], d.tb[k], m->W.tb[k], d.tb[k - 1], LoadSilu{ain, d.tb[k - 1]},
                    EpTwobodyOut{pre, ws_ptr<float>(ws, L.x[0]), geo, d.tb[k]});
      else
        sgemm<true>(st, rr, E, d.tb[k - 1], d.tb[k], m->W.tb[k], d.tb[k - 1], LoadSilu{ain, d.tb[k - 1]},
                    EpStore{pre, d.tb[k]});
    }
    sgemm<true>(st, rr, E, d.w, cw, m->W.env[0], d.w, LoadPlain{ws_ptr<float>(ws, L.x[0]), d.w},
                EpStore{ws_ptr<float>(ws, L.omega[0]), cw});
    AFM_LAUNCH_CHECK();
  }
  for (int layer = 1; layer <= d.NL; ++layer) {
    {
      int rc = tensor_products(m, ws, L, rr, layer, false, s.N, st);
      if (rc) return rc;
    }
    if (fused_last && layer == d.NL) {
      // forward and adjoint of the last layer; the adjoint's dE/dY
      // accumulators start here instead of in the backward
      int rc = zero_async(ws_ptr<float>(ws, L.gy), E * 64, st);
      if (!rc && d.lmax == 3) rc = zero_async(ws_ptr<float>(ws, L.gy3), E * GEO3_STRIDE * 4, st);
      if (rc) return rc;
      TraceScope tr(st, "latent_fb", layer);
      rc = mfma_latent_fb(m, ws, L, rr, s.species, s.seg, s.B, nullptr, st);
      if (rc) return rc;
      continue;
    }
    TraceScope tr(st, "latent_fwd", layer);
    if (m->prec == AFM_BF16_MFMA) {
      int rc = mfma_latent_fwd(m, ws, L, rr, layer, st);
      if (rc) return rc;
      continue;
    }
    const LayerPlan& lp = P.layer[layer - 1];
    const int ls = lp.n0e * d.c;
    const float* xprev = ws_ptr<float>(ws, L.x[layer - 1]);
    float* xnew = layer < d.NL ? ws_ptr<float>(ws, L.x[layer]) : ws_ptr<float>(ws, L.gt0);
    for (int k = 0; k < d.depth; ++k) {
      float* pre = ws_ptr<float>(ws, L.lat_pre[layer - 1][k]);
      const int kin = k == 0 ? d.w + ls : d.w;
      const bool last = k == d.depth - 1;
      if (k == 0) {
        LoadCat al{xprev, d.w, ws_ptr<float>(ws, L.s[layer - 1]), ls};
        if (last)
          sgemm<true>(st, rr, E, kin, d.w, m->W.lat[layer - 1][k], kin, al, EpLatentOut{pre, xprev, xnew, geo, d.w});
        else
          sgemm<true>(st, rr, E, kin, d.w, m->W.lat[layer - 1][k], kin, al, EpStore{pre, d.w});
      } else {
        LoadSilu al{ws_ptr<float>(ws, L.lat_pre[layer - 1][k - 1]), d.w};
        if (last)
          sgemm<true>(st, rr, E, kin, d.w, m->W.lat[layer - 1][k], kin, al, EpLatentOut{pre, xprev, xnew, geo, d.w});
        else
          sgemm<true>(st, rr, E, kin, d.w, m->W.lat[layer - 1][k], kin, al, EpStore{pre, d.w});
      }
    }
    if (layer < d.NL) {
      sgemm<true>(st, rr, E, d.w, cw, m->W.env[layer], d.w, LoadPlain{xnew, d.w},
                  EpStore{ws_ptr<float>(ws, L.omega[layer]), cw});
    } else {
      hipLaunchKernelGGL(k_edge_energy, dim3(grid_for(E, 4, 16384)), dim3(256), 0, st, rr, (const float*)xnew,
                         d.w, m->W.w_eff, ws_ptr<float>(ws, L.eps));
    }
    AFM_LAUNCH_CHECK();
  }
  return AFM_OK;
}

int run_backward_chunk(const afm_model* m, const SysDev& s, const NlDev& nl, const afm_workspace* ws,
                       const WsLayout& L, int chunk, const double* grad_e_struct, hipStream_t st, bool fused_last) {
  const ModelDims& d = m->dims;
  const Plan& P = m->plan;
  RowRange rr = row_range(nl, ws, L, chunk);
  const int64_t E = L.cex;
  float* geo = ws_ptr<float>(ws, L.geo);
  int32_t* eidx = ws_ptr<int32_t>(ws, L.eidx);
  float* gx = ws_ptr<float>(ws, L.gx);
  float* gt0 = ws_ptr<float>(ws, L.gt0);
  float* gt1 = ws_ptr<float>(ws, L.gt1);
  float* gy = ws_ptr<float>(ws, L.gy);
  const int cw = (d.lmax + 1) * d.c;
  int rc = AFM_OK;
  if (!fused_last) {   // (the fused last layer zeroed them and added its share)
    rc = zero_async(gy, E * 64, st);
    if (!rc && d.lmax == 3) rc = zero_async(ws_ptr<float>(ws, L.gy3), E * GEO3_STRIDE * 4, st);
  }
  if (rc) return rc;
  for (int layer = d.NL; layer >= 1; --layer) {
    const LayerPlan& lp = P.layer[layer - 1];
    const int ls = lp.n0e * d.c;
    if (!(fused_last && layer == d.NL)) {
      TraceScope tr(st, "latent_bwd", layer);
      if (m->prec == AFM_BF16_MFMA) {
        rc = mfma_latent_bwd(m, ws, L, rr, layer, s.species, s.seg, s.B, grad_e_struct, st);
        if (rc) return rc;
      } else {
        if (layer == d.NL) {
          hipLaunchKernelGGL(k_gx_init, dim3(grid_for(E * d.w, 256, 65536)), dim3(256), 0, st, rr,
                             (const int32_t*)eidx, s.species, s.seg, s.B, grad_e_struct, m->W.sp_scale, d.S,
                             d.escale, m->W.w_eff, d.w, gx);
        } else {
          // dE/dx^L += dE/domega^{L+1} W_env^{L+1}
          sgemm<false>(st, rr, E, cw, d.w, m->W.env[layer], d.w, LoadPlain{ws_ptr<float>(ws, L.gomega), cw},
                       EpAdd{gx, d.w});
        }
        AFM_LAUNCH_CHECK();
        // head: x^L = (x^{L-1} + u silu(a_D)) / sqrt 2
        const float r2 = 0.70710678118654752f;
        float* ga = gt0;
        hipLaunchKernelGGL(k_mlp_head_bwd, dim3(grid_for(E, 4, 16384)), dim3(256), 0, st, rr, d.w,
                           (const float*)ws_ptr<float>(ws, L.lat_pre[layer - 1][d.depth - 1]), (const float*)geo,
                           r2, r2, gx, ga, gy);
        AFM_LAUNCH_CHECK();
        for (int k = d.depth - 1; k >= 1; --k) {
          float* gnext = (ga == gt0) ? gt1 : gt0;
          sgemm<false>(st, rr, E, d.w, d.w, m->W.lat[layer - 1][k], d.w, LoadPlain{ga, d.w},
                       EpDsilu{ws_ptr<float>(ws, L.lat_pre[layer - 1][k - 1]), gnext, d.w});
          ga = gnext;
        }
        sgemm<false>(st, rr, E, d.w, d.w + ls, m->W.lat[layer - 1][0], d.w + ls, LoadPlain{ga, d.w},
                     EpSplit{gx, d.w, ws_ptr<float>(ws, L.gs[layer - 1]), ls});
        AFM_LAUNCH_CHECK();
      }
    }
    rc = tensor_products(m, ws, L, rr, layer, true, s.N, st);
    if (rc) return rc;
  }
  // two-body: dE/dx^0 += dE/domega^1 W_env^1, then the MLP adjoint
  {
    TraceScope tr(st, "twobody_bwd");
    if (m->prec == AFM_BF16_MFMA) {
      rc = mfma_twobody_bwd(m, ws, L, rr, s.species, st);
      if (rc) return rc;
    } else {
      sgemm<false>(st, rr, E, cw, d.w, m->W.env[0], d.w, LoadPlain{ws_ptr<float>(ws, L.gomega), cw},
                   EpAdd{gx, d.w});
      const int F = d.tb[d.ntb - 1];
      float* ga = gt0;
      hipLaunchKernelGGL(k_mlp_head_bwd, dim3(grid_for(E, 4, 16384)), dim3(256), 0, st, rr, F,
                         (const float*)ws_ptr<float>(ws, L.tb_pre[d.ntb - 1]), (const float*)geo, 1.0f, 0.0f, gx,
                         ga, gy);
      for (int k = d.ntb - 1; k >= 1; --k) {
        float* gnext = (ga == gt0) ? gt1 : gt0;
        sgemm<false>(st, rr, E, d.tb[k], d.tb[k - 1], m->W.tb[k], d.tb[k - 1], LoadPlain{ga, d.tb[k]},
                     EpDsilu{ws_ptr<float>(ws, L.tb_pre[k - 1]), gnext, d.tb[k - 1]});
        ga = gnext;
      }
      // dE/drho_n = sum_f ga[f] W_0[f][2S + n]
      sgemm<false>(st, rr, E, d.tb[0], d.nb, m->W.tb[0] + 2 * d.S, 2 * d.S + d.nb, LoadPlain{ga, d.tb[0]},
                   EpStore{ws_ptr<float>(ws, L.grho), 16});
      AFM_LAUNCH_CHECK();
    }
  }
  TraceScope tr(st, "geometry_bwd");
  hipLaunchKernelGGL(k_geometry_bwd, dim3(grid_for(E, 256, 65536)), dim3(256), 0, st, rr, (const float*)geo,
                     (const float*)ws_ptr<float>(ws, L.grho), (const float*)gy,
                     d.lmax == 3 ? (const float*)ws_ptr<float>(ws, L.gy3) : nullptr, d.nb, (float)d.r_cut, d.p,
                     ws_ptr<float>(ws, L.g));
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

int run_atom_energy(const afm_model* m, const SysDev& s, const NlDev& nl, const afm_workspace* ws,
                    const WsLayout& L, double* e_atom, double* e_struct, hipStream_t st) {
  TraceScope tr(st, "energy");
  hipLaunchKernelGGL(k_atom_energy, dim3(grid_for(s.N * kRowLanes, kRowBlock)), dim3(kRowBlock), 0, st, (const int64_t*)nl.row_ptr, s.N,
                     nl.capacity, (const float*)ws_ptr<float>(ws, L.eps), s.species, m->dims.S, m->W.sp_scale,
                     m->W.sp_shift, m->dims.escale, e_atom, nl.status);
  if (e_struct)
    hipLaunchKernelGGL(k_struct_sum<1>, dim3((unsigned)s.B), dim3(kSumBlock), 0, st, s.seg, (const double*)e_atom,
                       e_struct);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

int run_force_scatter(const afm_model* m, const SysDev& s, const NlDev& nl, const afm_workspace* ws,
                      const WsLayout& L, double* forces, double* virial, hipStream_t st) {
  TraceScope tr(st, "force_scatter");
  double* wat = virial ? ws_ptr<double>(ws, L.atom_virial) : nullptr;
  hipLaunchKernelGGL(k_force_scatter, dim3(grid_for(s.N * kRowLanes, kRowBlock)), dim3(kRowBlock), 0, st, s.pos, s.cell, s.pbc, s.seg,
                     s.B, (const int64_t*)nl.row_ptr, s.N, (const int32_t*)nl.col, (const int8_t*)nl.shift,
                     (const int32_t*)nl.rev, (const float*)ws_ptr<float>(ws, L.g), nl.capacity, forces, wat);
  if (virial)
    hipLaunchKernelGGL(k_struct_sum<9>, dim3((unsigned)s.B), dim3(kSumBlock), 0, st, s.seg, (const double*)wat, virial);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

// out_i = sum_{e in row i} (g_e - g_rev(e)) for a per-edge vector field g
// [capacity][3] (the force scatter without virials)
int run_edge_scatter(const SysDev& s, const NlDev& nl, const float* g, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_force_scatter, dim3(grid_for(s.N * kRowLanes, kRowBlock)), dim3(kRowBlock), 0, st, s.pos, s.cell,
                     s.pbc, s.seg, s.B, (const int64_t*)nl.row_ptr, s.N, (const int32_t*)nl.col,
                     (const int8_t*)nl.shift, (const int32_t*)nl.rev, g, nl.capacity, out, (double*)nullptr);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

}  // namespace afm
