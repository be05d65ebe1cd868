// Backward of the force adjoint: weight gradients for force matching
// (Methodology / Model Training: the loss combines energy and force errors,
// so training needs d/dtheta of the forces).
//
// Objective J(theta) = sum_s gE_s E_s + sum_i gF_i . F_i + sum_s gW_s : W_s.
// With F_i = -dE/dr_i and W_s = -sum_e g_e delta_e^T (g_e = dE/d delta_e)
// this is J = sum_s gE_s E_s - Edot, where Edot is the derivative of E along
// the edge tangents delta_dot_e = (gF_j - gF_i) + gW_s delta_e: positions
// moving with velocity gF plus a homogeneous deformation gW of each
// structure (the stress term).  The schedule is forward-over-reverse:
// every network quantity z gets a tangent z_dot (stacked as extra rows under
// the primal rows, so each GEMM serves both), then J is reversed with
// respect to the weights through primal and tangent together.  Basis and
// spherical harmonics (and their tangents) do not depend on the weights, so
// the weight gradient needs no second derivatives of the geometry.  The
// optional position gradient dJ/dr does: the reverse also collects, per
// edge, the adjoints of the basis b = (rho_n, u, Y) and of its tangent b_dot
// (primal and tangent rows), and a per-edge kernel differentiates
// phi(delta, delta_dot) = b_bar . b + b_dot_bar . b_dot by forward-mode
// dual numbers in delta and in delta_dot (delta_dot = (gF_j - gF_i) +
// gW delta also depends on delta).  The per-edge results are scattered to
// the atoms like forces.  Everything runs in FP32:
// the GEMMs and weight-gradient reductions on the matrix cores
// (v_mfma_f32_16x16x4f32), the tensor products on the vector ALUs over the
// CG nonzeros; weight gradients are reduced in fixed-order slices and
// accumulated in FP64 (deterministic).  Chunks of rows are exact (E_i and
// Edot_i depend only on row i).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "cg_ct.h"
#include "device_util.h"
#include "edge_layout.h"
#include "gemm_f32.h"
#include "internal.h"
#include "trace.h"

namespace afm {

// weight gradients reduce over edge rows in slices summed afterwards in a
// fixed order; enough slices that a launch has ~1024 workgroups
constexpr int kMaxSlices = 256;
// per-edge basis adjoints for the position gradient: [row][kBadj] with
// [0..8] Y, [9] u, [16 + n] rho_n (rows t primal, stack + t tangent)
constexpr int kBadj = 32;

__device__ __forceinline__ float sig_f(float a) { return 1.0f / (1.0f + expf(-a)); }
__device__ __forceinline__ float d1silu(float a) {
  const float s = sig_f(a);
  return s * (1.0f + a * (1.0f - s));
}
// silu''(a) = s (1 - s) (2 + a (1 - 2 s))
__device__ __forceinline__ float d2silu(float a) {
  const float s = sig_f(a);
  return s * (1.0f - s) * (2.0f + a * (1.0f - 2.0f * s));
}

__device__ __forceinline__ float env_f(float x, int p) {
  if (x >= 1.0f) return 0.0f;
  float xp = 1.0f;
  for (int q = 0; q < p; ++q) xp *= x;
  return 1.0f - 0.5f * (p + 1) * (p + 2) * xp + (float)(p * (p + 2)) * xp * x - 0.5f * p * (p + 1) * xp * x * x;
}
__device__ __forceinline__ float env_dx_f(float x, int p) {
  if (x >= 1.0f) return 0.0f;
  float xp = 1.0f;
  for (int q = 0; q < p - 1; ++q) xp *= x;
  return -0.5f * p * (p + 1) * (p + 2) * xp * (1.0f - x) * (1.0f - x);
}

// forward derivative of the 9 harmonics at unit u along w
__device__ __forceinline__ void sh9_jvp(float x, float y, float z, const float* w, float* Yd) {
  const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s5h = 1.118033988749895f;
  Yd[0] = 0.0f;
  Yd[1] = s3 * w[1]; Yd[2] = s3 * w[2]; Yd[3] = s3 * w[0];
  Yd[4] = s15 * (x * w[1] + y * w[0]);
  Yd[5] = s15 * (y * w[2] + z * w[1]);
  Yd[6] = s5h * 6.0f * z * w[2];
  Yd[7] = s15 * (x * w[2] + z * w[0]);
  Yd[8] = s15 * (x * w[0] - y * w[1]);
}

// ----------------------------------------------------------------------------
// position gradient: dual numbers (a value and its gradient with respect to
// three seeded inputs) through the edge basis and its tangent

struct D3 {
  float v, g[3];
};
__device__ __forceinline__ D3 dc(float v) { return D3{v, {0.0f, 0.0f, 0.0f}}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return D3{a.v + b.v, {a.g[0] + b.g[0], a.g[1] + b.g[1], a.g[2] + b.g[2]}}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return D3{a.v - b.v, {a.g[0] - b.g[0], a.g[1] - b.g[1], a.g[2] - b.g[2]}}; }
__device__ __forceinline__ D3 operator*(D3 a, D3 b) {
  return D3{a.v * b.v, {a.g[0] * b.v + a.v * b.g[0], a.g[1] * b.v + a.v * b.g[1], a.g[2] * b.v + a.v * b.g[2]}};
}
__device__ __forceinline__ D3 operator*(float s, D3 a) { return D3{s * a.v, {s * a.g[0], s * a.g[1], s * a.g[2]}}; }
__device__ __forceinline__ D3 operator*(D3 a, float s) { return s * a; }
__device__ __forceinline__ D3 operator+(float s, D3 a) { return D3{s + a.v, {a.g[0], a.g[1], a.g[2]}}; }
// a function f of a dual: f(a.v) and chain rule with f'(a.v)
__device__ __forceinline__ D3 dapply(D3 a, float f, float df) {
  return D3{f, {df * a.g[0], df * a.g[1], df * a.g[2]}};
}
__device__ __forceinline__ D3 drcp(D3 a) {
  const float r = 1.0f / a.v;
  return dapply(a, r, -r * r);
}
__device__ __forceinline__ D3 dsqrt(D3 a) {
  const float s = sqrtf(a.v);
  return dapply(a, s, 0.5f / s);
}
__device__ __forceinline__ D3 dpow(D3 a, int n) {
  D3 r = dc(1.0f);
  for (int q = 0; q < n; ++q) r = r * a;
  return r;
}
// polynomial envelope u(x) and its derivative du/dx, x = d / r_c < 1
__device__ __forceinline__ D3 denv(D3 x, int p) {
  const D3 xp = dpow(x, p);
  return 1.0f + ((-0.5f * (p + 1) * (p + 2)) * xp + (float)(p * (p + 2)) * (xp * x) +
                 (-0.5f * p * (p + 1)) * (xp * x * x));
}
__device__ __forceinline__ D3 denv_dx(D3 x, int p) {
  const D3 omx = 1.0f + (-1.0f) * x;
  return (-0.5f * p * (p + 1) * (p + 2)) * (dpow(x, p - 1) * omx * omx);
}

// phi = sum_k bbar_k b_k + bdbar_k b_dot_k over the edge basis b = (rho_n
// (n < nb), u, Y (9)) and its tangent along delta_dot, evaluated with dual
// inputs; bbar / bdbar: [0..8] Y, [9] u, [16 + n] rho_n.  Mirrors the basis
// of the forward kernels: rho_n = B_n(d) u(d), B_n = sqrt(2/r_c) sin(k_n d)/d,
// Y = sh9(delta/d), u_dot = u'(d) d_dot, Y_dot = the forward derivative of
// Y along (delta_dot - u d_dot)/d.
__device__ D3 basis_phi(const D3* dl, const D3* dd, float r_cut, int p, int nb, const float* bbar,
                        const float* bdbar) {
  const D3 r = dsqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
  const D3 inv = drcp(r);
  const D3 ux = dl[0] * inv, uy = dl[1] * inv, uz = dl[2] * inv;
  const D3 rd = ux * dd[0] + uy * dd[1] + uz * dd[2];
  const D3 wx = (dd[0] - ux * rd) * inv, wy = (dd[1] - uy * rd) * inv, wz = (dd[2] - uz * rd) * inv;
  D3 phi = dc(0.0f);
  const D3 x = (1.0f / r_cut) * r;
  if (x.v < 1.0f) {
    const D3 u = denv(x, p);
    const D3 up = (1.0f / r_cut) * denv_dx(x, p);
    phi = phi + bbar[9] * u + bdbar[9] * (up * rd);
    const float c = sqrtf(2.0f / r_cut);
    for (int n = 0; n < nb; ++n) {
      const float k = (n + 1) * 3.14159265358979323846f / r_cut;
      const D3 kr = k * r;
      const D3 sn = dapply(kr, sinf(kr.v), cosf(kr.v));
      const D3 cs = dapply(kr, cosf(kr.v), -sinf(kr.v));
      const D3 B = c * (sn * inv);
      const D3 dB = c * ((k * cs) * inv + (-1.0f) * (sn * inv * inv));
      phi = phi + bbar[16 + n] * (B * u) + bdbar[16 + n] * ((dB * u + B * up) * rd);
    }
  }
  const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s5h = 1.118033988749895f;
  // Y without its constant parts (Y_0 = 1 and the -1 of Y_6): only the
  // gradient of phi is used
  D3 yv = bbar[1] * (s3 * uy) + bbar[2] * (s3 * uz) + bbar[3] * (s3 * ux);
  yv = yv + bbar[4] * (s15 * (ux * uy)) + bbar[5] * (s15 * (uy * uz)) + bbar[6] * (s5h * (3.0f * (uz * uz)));
  yv = yv + bbar[7] * (s15 * (ux * uz)) + bbar[8] * ((0.5f * s15) * (ux * ux + (-1.0f) * (uy * uy)));
  // Y_dot
  D3 ydv = bdbar[1] * (s3 * wy) + bdbar[2] * (s3 * wz) + bdbar[3] * (s3 * wx);
  ydv = ydv + bdbar[4] * (s15 * (ux * wy + uy * wx)) + bdbar[5] * (s15 * (uy * wz + uz * wy));
  ydv = ydv + bdbar[6] * ((6.0f * s5h) * (uz * wz)) + bdbar[7] * (s15 * (ux * wz + uz * wx));
  ydv = ydv + bdbar[8] * (s15 * (ux * wx + (-1.0f) * (uy * wy)));
  return phi + yv + ydv;
}

// tangent geometry: geo2[t] = (delta_dot[3], d_dot, u_dot, Y_dot[9], -, -)
__global__ void k_geom2(RowRange rr, const float* __restrict__ geo, const int32_t* __restrict__ eidx,
                        const int32_t* __restrict__ col, const double* __restrict__ gF,
                        const double* __restrict__ gW, const int64_t* __restrict__ seg, int64_t B, float r_cut,
                        int p, float* __restrict__ geo2) {
  int64_t e0, e1;
  rr.get(e0, e1);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < e1 - e0; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = eidx[t], j = col[e0 + t];
    const float* G = geo + t * GEO_STRIDE;
    double dd64[3] = {0.0, 0.0, 0.0};
    if (gF)
      for (int q = 0; q < 3; ++q) dd64[q] = gF[3 * j + q] - gF[3 * i + q];
    if (gW) {
      int64_t lo = 0, hi = B;
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (seg[mid] <= i) lo = mid; else hi = mid;
      }
      const double* w = gW + 9 * lo;
      for (int q = 0; q < 3; ++q)
        dd64[q] += w[3 * q] * (double)G[0] + w[3 * q + 1] * (double)G[1] + w[3 * q + 2] * (double)G[2];
    }
    float dd[3];
    for (int q = 0; q < 3; ++q) dd[q] = (float)dd64[q];
    const float r = G[GEO_D];
    float* o = geo2 + t * GEO_STRIDE;
    if (r > 0.0f) {
      const float inv = 1.0f / r;
      const float u[3] = {G[0] * inv, G[1] * inv, G[2] * inv};
      const float rd = u[0] * dd[0] + u[1] * dd[1] + u[2] * dd[2];
      const float w[3] = {(dd[0] - u[0] * rd) * inv, (dd[1] - u[1] * rd) * inv, (dd[2] - u[2] * rd) * inv};
      float Yd[9];
      sh9_jvp(u[0], u[1], u[2], w, Yd);
      o[0] = dd[0]; o[1] = dd[1]; o[2] = dd[2];
      o[GEO_D] = rd;
      o[GEO_U] = env_dx_f(r / r_cut, p) / r_cut * rd;
      for (int q = 0; q < 9; ++q) o[GEO_Y + q] = Yd[q];
    } else {
      for (int q = 0; q < 14; ++q) o[q] = 0.0f;
    }
    o[14] = 0.0f; o[15] = 0.0f;
  }
}

// rho_n and its tangent for edge t
__device__ __forceinline__ void rho_pair(const float* G, const float* G2, float r_cut, int p, int n, float& rho,
                                         float& rhod) {
  const float r = G[GEO_D], u = G[GEO_U];
  const float c = sqrtf(2.0f / r_cut);
  const float k = (n + 1) * 3.14159265358979323846f / r_cut;
  const float sn = sinf(k * r), cs = cosf(k * r);
  const float B = c * sn / r;
  const float dB = c * (k * cs / r - sn / (r * r));
  const float du = env_dx_f(r / r_cut, p) / r_cut;
  rho = B * u;
  rhod = (dB * u + B * du) * G2[GEO_D];
}

// first two-body layer, primal rows t and tangent rows stack + t
__global__ void k_tb2_first(RowRange rr, int stack, const float* __restrict__ geo, const float* __restrict__ geo2,
                            const int32_t* __restrict__ eidx, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ species, const float* __restrict__ W, int S, int nb, int F,
                            float r_cut, int p, float* __restrict__ pre) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  const int K = 2 * S + nb;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < M * F; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / F;
    const int f = (int)(q % F);
    const int zi = min(max(species[eidx[t]], 0), S - 1), zj = min(max(species[col[e0 + t]], 0), S - 1);
    const float* w = W + (int64_t)f * K;
    float a = w[zi] + w[S + zj], ad = 0.0f;
    for (int n = 0; n < nb; ++n) {
      float rho, rhod;
      rho_pair(geo + t * GEO_STRIDE, geo2 + t * GEO_STRIDE, r_cut, p, n, rho, rhod);
      a += w[2 * S + n] * rho;
      ad += w[2 * S + n] * rhod;
    }
    pre[t * F + f] = a;
    pre[(stack + t) * F + f] = ad;
  }
}

// x0 = u silu(a), x0_dot = u_dot silu(a) + u silu'(a) a_dot
__global__ void k_tb2_out(RowRange rr, int stack, int F, const float* __restrict__ pre,
                          const float* __restrict__ geo, const float* __restrict__ geo2, float* __restrict__ x) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < M * F; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / F;
    const int f = (int)(q % F);
    const float a = pre[t * F + f], ad = pre[(stack + t) * F + f];
    const float u = geo[t * GEO_STRIDE + GEO_U], ud = geo2[t * GEO_STRIDE + GEO_U];
    x[t * F + f] = u * a * sig_f(a);
    x[(stack + t) * F + f] = ud * a * sig_f(a) + u * d1silu(a) * ad;
  }
}

// x^L = (x^{L-1} + u silu(a)) / sqrt 2 and its tangent
__global__ void k_lat2_out(RowRange rr, int stack, int F, const float* __restrict__ pre,
                           const float* __restrict__ xprev, const float* __restrict__ geo,
                           const float* __restrict__ geo2, float* __restrict__ x) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  const float r2 = 0.70710678118654752f;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < M * F; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / F;
    const int f = (int)(q % F);
    const float a = pre[t * F + f], ad = pre[(stack + t) * F + f];
    const float u = geo[t * GEO_STRIDE + GEO_U], ud = geo2[t * GEO_STRIDE + GEO_U];
    const float h = a * sig_f(a), hd = d1silu(a) * ad;
    x[t * F + f] = (xprev[t * F + f] + u * h) * r2;
    x[(stack + t) * F + f] = (xprev[(stack + t) * F + f] + ud * h + u * hd) * r2;
  }
}

__device__ __forceinline__ int64_t struct_of(const int64_t* seg, int64_t B, int64_t i) {
  int64_t lo = 0, hi = B;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (seg[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// eps, eps_dot, the initial adjoints of x^{N_L} and the coefficients used
// for the edge-energy weight gradient
__global__ void __launch_bounds__(256) k_energy2(RowRange rr, int stack, int w, const float* __restrict__ x,
                                                 const float* __restrict__ w_eff, const int32_t* __restrict__ eidx,
                                                 const int32_t* __restrict__ species, const double* __restrict__ sc,
                                                 int S, double escale, const int64_t* __restrict__ seg, int64_t B,
                                                 const double* __restrict__ gE, float* __restrict__ eps2,
                                                 float* __restrict__ coef, float* __restrict__ gx) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  const int lane = threadIdx.x & 63;
  for (int64_t t = blockIdx.x * 4 + (threadIdx.x >> 6); t < M; t += (int64_t)gridDim.x * 4) {
    const int64_t i = eidx[t];
    const float cs = (float)(sc[min(max(species[i], 0), S - 1)] * escale);
    const float ge = gE ? (float)gE[struct_of(seg, B, i)] : 0.0f;
    float a = 0.0f, ad = 0.0f;
    for (int f = lane; f < w; f += 64) {
      a += w_eff[f] * x[t * w + f];
      ad += w_eff[f] * x[(stack + t) * w + f];
      gx[t * w + f] = ge * cs * w_eff[f];
      gx[(stack + t) * w + f] = -cs * w_eff[f];
    }
    a = group_sum<64>(a);
    ad = group_sum<64>(ad);
    if (lane == 0) {
      eps2[t] = a;
      eps2[stack + t] = ad;
      coef[t] = ge * cs;
      coef[stack + t] = -cs;
    }
  }
}

// per-atom shares of the species-scale and species-shift gradients
__global__ void k_atom2(RowRange rr, int stack, const float* __restrict__ eps2, const int32_t* __restrict__ species,
                        int S, double escale, const int64_t* __restrict__ seg, int64_t B,
                        const double* __restrict__ gE, double* __restrict__ a_sig, double* __restrict__ a_mu) {
  const int64_t a0 = rr.chunk_rows[rr.chunk], a1 = rr.chunk_rows[rr.chunk + 1];
  const int64_t e0 = rr.row_ptr[a0];
  for (int64_t i = a0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a1; i += (int64_t)gridDim.x * blockDim.x) {
    double se = 0.0, sd = 0.0;
    for (int64_t e = rr.row_ptr[i]; e < rr.row_ptr[i + 1]; ++e) {
      se += (double)eps2[e - e0];
      sd += (double)eps2[stack + e - e0];
    }
    const double ge = gE ? gE[struct_of(seg, B, i)] : 0.0;
    a_sig[i] = escale * (ge * se - sd);
    a_mu[i] = ge;
  }
}

// h = silu(a) (rows t) and h_dot = silu'(a) a_dot (rows stack + t) of the
// stacked pre-activations, written once for the GEMMs that read them (a
// loader that applied them would do so once per output-column tile)
__global__ void k_act2_fwd(RowRange rr, int stack, int F, const float* __restrict__ pre, float* __restrict__ out) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < M * F; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / F;
    const int f = (int)(q % F);
    const float a = pre[t * F + f];
    out[t * F + f] = silu_f(a);
    out[(stack + t) * F + f] = d1silu(a) * pre[(stack + t) * F + f];
  }
}

// the concatenated first-GEMM input [x | s] of the stacked rows, written
// once for the GEMM that reads it
__global__ void k_cat2(RowRange rr, int stack, const float* __restrict__ x, int w, const float* __restrict__ sv, int ls,
                       float* __restrict__ out) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  const int F = w + ls;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < M * F; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / F;
    const int f = (int)(q % F);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r = t + h * (int64_t)stack;
      out[r * F + f] = f < w ? x[r * w + f] : sv[r * ls + (f - w)];
    }
  }
}

// adjoint through an activation: given dJ/dh (rows t) and dJ/dh_dot
// (rows stack + t) with h = silu(a), h_dot = silu'(a) a_dot:
//   a_bar = h_bar silu'(a) + hd_bar silu''(a) a_dot;  ad_bar = hd_bar silu'(a)
// head = 1: the input is the adjoint of y = s (x_prev + u h) with s = r2
// (latent) or y = u h with no residual (two-body, res = 0); it then also
// scales the residual share in place.
__global__ void k_act2_bwd(RowRange rr, int stack, int F, const float* __restrict__ pre, float* __restrict__ gin,
                           float* __restrict__ gout, const float* __restrict__ geo, const float* __restrict__ geo2,
                           int head, float scale, float res) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < M * F; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / F;
    const int f = (int)(q % F);
    const float a = pre[t * F + f], ad = pre[(stack + t) * F + f];
    float hb = gin[t * F + f], hdb = gin[(stack + t) * F + f];
    if (head) {
      const float u = geo[t * GEO_STRIDE + GEO_U], ud = geo2[t * GEO_STRIDE + GEO_U];
      const float xb = hb * scale, xdb = hdb * scale;
      gin[t * F + f] = hb * res;
      gin[(stack + t) * F + f] = hdb * res;
      hb = u * xb + ud * xdb;
      hdb = u * xdb;
    }
    gout[t * F + f] = hb * d1silu(a) + hdb * d2silu(a) * ad;
    gout[(stack + t) * F + f] = hdb * d1silu(a);
  }
}

// Position gradient, u adjoints: for the head y = s (x_prev + u h) (latent,
// s = r2) or y = u h (two-body, s = 1) with h = silu(a), and its tangent
// y_dot = s (x_prev_dot + u_dot h + u h_dot), given dJ/dy (rows t) and
// dJ/dy_dot (rows stack + t) before k_act2_bwd rewrites them:
//   dJ/du += s sum_f (ybar h + ydbar h_dot);  dJ/du_dot += s sum_f ydbar h.
// One wavefront per edge.
__global__ void __launch_bounds__(256) k_u2_adj(RowRange rr, int stack, int F, const float* __restrict__ pre,
                                               const float* __restrict__ gin, float scale, float* __restrict__ badj) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  const int lane = threadIdx.x & 63;
  for (int64_t t = blockIdx.x * 4 + (threadIdx.x >> 6); t < M; t += (int64_t)gridDim.x * 4) {
    const int64_t ts = stack + t;
    float su = 0.0f, sud = 0.0f;
    for (int f = lane; f < F; f += 64) {
      const float a = pre[t * F + f], ad = pre[ts * F + f];
      const float yb = gin[t * F + f], ydb = gin[ts * F + f];
      const float h = a * sig_f(a), hd = d1silu(a) * ad;
      su += yb * h + ydb * hd;
      sud += ydb * h;
    }
    su = group_sum<64>(su);
    sud = group_sum<64>(sud);
    if (lane == 0) {
      badj[t * kBadj + 9] += scale * su;
      badj[ts * kBadj + 9] += scale * sud;
    }
  }
}

// rho adjoints from the first two-body layer a0 = W0 [onehot | onehot | rho],
// a0_dot = W0_rho rho_dot:  dJ/drho_n = sum_f ga[t][f] W0[f][2S + n] (and
// the same on the tangent rows).  One thread per (row, n).
__global__ void k_rho2_adj(RowRange rr, int stack, const float* __restrict__ ga, const float* __restrict__ W0,
                           int S, int nb, int T0, float* __restrict__ badj) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  const int K = 2 * S + nb;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < 2 * M * nb;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(q % nb);
    const int64_t rt = q / nb;
    const int64_t row = rt < M ? rt : stack + (rt - M);
    float v = 0.0f;
    for (int f = 0; f < T0; ++f) v += ga[row * T0 + f] * W0[(int64_t)f * K + 2 * S + n];
    badj[row * kBadj + 16 + n] = v;
  }
}

// dJ/d delta_e = d phi/d delta + gW^T d phi/d delta_dot (phi: basis_phi),
// written at the edge's global index.
__global__ void k_gpos_edge(RowRange rr, int stack, const float* __restrict__ geo, const float* __restrict__ geo2,
                            const float* __restrict__ badj, const int32_t* __restrict__ eidx,
                            const double* __restrict__ gW, const int64_t* __restrict__ seg, int64_t B, float r_cut,
                            int p, int nb, float* __restrict__ gpos_e) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int64_t M = e1 - e0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < M; t += (int64_t)gridDim.x * blockDim.x) {
    const float* G = geo + t * GEO_STRIDE;
    const float* G2 = geo2 + t * GEO_STRIDE;
    float res[3] = {0.0f, 0.0f, 0.0f};
    if (G[GEO_D] > 0.0f) {
      const float* bb = badj + t * kBadj;
      const float* bd = badj + (stack + t) * kBadj;
      D3 dl[3], dd[3];
      // d/d delta (delta_dot held)
      for (int q = 0; q < 3; ++q) {
        dl[q] = dc(G[q]);
        dl[q].g[q] = 1.0f;
        dd[q] = dc(G2[q]);
      }
      const D3 a = basis_phi(dl, dd, r_cut, p, nb, bb, bd);
      // d/d delta_dot (delta held)
      for (int q = 0; q < 3; ++q) {
        dl[q] = dc(G[q]);
        dd[q] = dc(G2[q]);
        dd[q].g[q] = 1.0f;
      }
      const D3 b = basis_phi(dl, dd, r_cut, p, nb, bb, bd);
      for (int q = 0; q < 3; ++q) res[q] = a.g[q];
      if (gW) {
        const double* w = gW + 9 * struct_of(seg, B, eidx[t]);
        // delta_dot_q += sum_c gW[q][c] delta_c  =>  d/d delta_c += gW[q][c] b_q
        for (int c = 0; c < 3; ++c)
          res[c] += (float)(w[c] * b.g[0] + w[3 + c] * b.g[1] + w[6 + c] * b.g[2]);
      }
    }
    for (int q = 0; q < 3; ++q) gpos_e[3 * (e0 + t) + q] = res[q];
  }
}

__global__ void k_negate_f64(double* __restrict__ a, int64_t n) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    a[q] = -a[q];
}

// ----------------------------------------------------------------------------
// tensor products with tangents

struct TP2Args {
  RowRange rr;
  int stack;
  const float* geo;
  const float* geo2;
  const float* omega;    // stacked omega^L
  const float* omega1;   // stacked omega^1
  const float* vin;      // stacked V^{L-1}
  float* vout;           // stacked V^L
  float* s;              // stacked s^L
  float* gamma;          // Gamma^L   [N][NLM][C]
  float* gammad;         // Gamma_dot [N][NLM][C]
  const float* alpha;
  float inv_sqrt_nbar;
  const float* gs;       // stacked dJ/ds
  const float* gvout;    // stacked dJ/dV^L
  float* gvin;           // stacked dJ/dV^{L-1}
  float* gomega;         // stacked dJ/domega^L
  float* galpha;         // [N][n_paths][C] per-atom alpha-gradient shares
  float* badj;           // position gradient: stacked per-edge basis adjoints (+= dJ/dY), or null
  int c0;                // first channel of this launch (the arrays hold CS channels)
};

// sum over the C channel lanes of one edge slot (lanes of a slot are
// contiguous), then lane n == 0 adds the 9 + 9 totals to the edge's Y and
// Y_dot adjoints
template <int C>
__device__ __forceinline__ void add_ybar(float* __restrict__ badj, int64_t t, int64_t ts, int n, float* yb,
                                         float* ydb) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    yb[q] = group_sum<C>(yb[q]);
    ydb[q] = group_sum<C>(ydb[q]);
  }
  if (n == 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      badj[t * kBadj + q] += yb[q];
      badj[ts * kBadj + q] += ydb[q];
    }
  }
}

template <int LMAX, int NL, int L>
struct LayerCT2 {
  static constexpr LayerPlan lp = PlanCT<LMAX, NL>::plan.layer[L - 1];
};

// the products of one path over the CG nonzeros (compile-time tables):
// T[m3] = sum C V[m1] G[m2] and its tangent Td = sum C (Vd G + V Gd)
template <int LMAX, int NL, int L, int K>
__device__ __forceinline__ void path2(const float* V, const float* Vd, const float* G, const float* Gd, float* T,
                                      float* Td) {
  constexpr PathT pt = LayerCT2<LMAX, NL, L>::lp.p[K];
  constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
#pragma unroll
  for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) { T[m3] = 0.0f; Td[m3] = 0.0f; }
  static_for<0, nz.n>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    const float v = V[pt.in_off + nz.m1[q]], vd = Vd[pt.in_off + nz.m1[q]];
    const float g = G[pt.l2 * pt.l2 + nz.m2[q]], gd = Gd[pt.l2 * pt.l2 + nz.m2[q]];
    T[nz.m3[q]] += nz.c[q] * v * g;
    Td[nz.m3[q]] += nz.c[q] * (vd * g + v * gd);
  });
}

template <int LMAX, int NL, int L, int CS>
__device__ __forceinline__ void load_V2(const TP2Args& a, int64_t t, int nc, const float* Y, const float* Yd, float* V,
                                        float* Vd) {
  constexpr LayerPlan LP = LayerCT2<LMAX, NL, L>::lp;
  const int64_t ts = a.stack + t;
  if constexpr (L == 1) {
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
      const float w = a.omega1[(t * (LMAX + 1) + l) * CS + nc];
      const float wd = a.omega1[(ts * (LMAX + 1) + l) * CS + nc];
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) {
        V[l * l + m] = w * Y[l * l + m];
        Vd[l * l + m] = wd * Y[l * l + m] + w * Yd[l * l + m];
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < LP.n_in_comps; ++q) {
      V[q] = a.vin[(t * LP.n_in_comps + q) * CS + nc];
      Vd[q] = a.vin[(ts * LP.n_in_comps + q) * CS + nc];
    }
  }
}

// C: channels per launch (the lanes of an edge slot); CS: channels in the
// arrays (128 channels run as two launches of 64)
template <int LMAX, int NL, int L, int C, int CS>
__global__ void __launch_bounds__(256) k_tp2_fwd(TP2Args a) {
  constexpr LayerPlan LP = LayerCT2<LMAX, NL, L>::lp;
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  constexpr int NS = 256 / C;
  constexpr int NCI = LP.n_in_comps, NCO = LP.n_out_comps > 0 ? LP.n_out_comps : 1;
  __shared__ float red[2 * NS * NLM * C];
  __shared__ float gam[NLM * C];
  __shared__ float gamd[NLM * C];
  const int n = threadIdx.x % C, slot = threadIdx.x / C;
  const int nc = a.c0 + n;   // channel in the arrays
  const int64_t a0 = a.rr.chunk_rows[a.rr.chunk], a1 = a.rr.chunk_rows[a.rr.chunk + 1];
  const int64_t e0 = a.rr.row_ptr[a0];
  for (int64_t i = a0 + blockIdx.x; i < a1; i += gridDim.x) {
    const int64_t eb = a.rr.row_ptr[i], ee = a.rr.row_ptr[i + 1];
    float acc[NLM], accd[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) { acc[q] = 0.0f; accd[q] = 0.0f; }
    for (int64_t e = eb + slot; e < ee; e += NS) {
      const int64_t t = e - e0, ts = a.stack + t;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
      const float* Yd = a.geo2 + t * GEO_STRIDE + GEO_Y;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        const float w = a.omega[(t * (LMAX + 1) + l) * CS + nc];
        const float wd = a.omega[(ts * (LMAX + 1) + l) * CS + nc];
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) {
          acc[l * l + m] += w * Y[l * l + m];
          accd[l * l + m] += wd * Y[l * l + m] + w * Yd[l * l + m];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      red[(slot * NLM + q) * C + n] = acc[q];
      red[((NS + slot) * NLM + q) * C + n] = accd[q];
    }
    __syncthreads();
    for (int q = slot; q < NLM; q += NS) {
      float g = 0.0f, gd = 0.0f;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        g += red[(s * NLM + q) * C + n];
        gd += red[((NS + s) * NLM + q) * C + n];
      }
      g *= a.inv_sqrt_nbar;
      gd *= a.inv_sqrt_nbar;
      gam[q * C + n] = g;
      gamd[q * C + n] = gd;
      a.gamma[(i * NLM + q) * CS + nc] = g;
      a.gammad[(i * NLM + q) * CS + nc] = gd;
    }
    __syncthreads();
    float G[NLM], Gd[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) { G[q] = gam[q * C + n]; Gd[q] = gamd[q * C + n]; }
    for (int64_t e = eb + slot; e < ee; e += NS) {
      const int64_t t = e - e0, ts = a.stack + t;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
      const float* Yd = a.geo2 + t * GEO_STRIDE + GEO_Y;
      float V[NCI], Vd[NCI];
      load_V2<LMAX, NL, L, CS>(a, t, nc, Y, Yd, V, Vd);
      float out[NCO], outd[NCO];
#pragma unroll
      for (int q = 0; q < NCO; ++q) { out[q] = 0.0f; outd[q] = 0.0f; }
      static_for<0, LP.n_paths>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr PathT pt = LP.p[k];
        constexpr int d3 = 2 * pt.l3 + 1;
        float T[d3], Td[d3];
        path2<LMAX, NL, L, k>(V, Vd, G, Gd, T, Td);
        if constexpr (pt.s_idx >= 0) {
          a.s[(t * LP.n0e + pt.s_idx) * CS + nc] = T[0];
          a.s[(ts * LP.n0e + pt.s_idx) * CS + nc] = Td[0];
        }
        if constexpr (pt.out_off >= 0) {
          const float al = a.alpha[k * CS + nc];
#pragma unroll
          for (int m3 = 0; m3 < d3; ++m3) {
            out[pt.out_off + m3] += al * T[m3];
            outd[pt.out_off + m3] += al * Td[m3];
          }
        }
      });
      if constexpr (LP.n_out_comps > 0) {
#pragma unroll
        for (int q = 0; q < LP.n_out_comps; ++q) {
          a.vout[(t * LP.n_out_comps + q) * CS + nc] = out[q];
          a.vout[(ts * LP.n_out_comps + q) * CS + nc] = outd[q];
        }
      }
    }
    __syncthreads();
  }
}

template <int LMAX, int NL, int L, int C, int CS>
__global__ void __launch_bounds__(256) k_tp2_bwd(TP2Args a) {
  constexpr LayerPlan LP = LayerCT2<LMAX, NL, L>::lp;
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  constexpr int NS = 256 / C;
  constexpr int NCI = LP.n_in_comps;
  constexpr int NP = LP.n_paths;
  __shared__ float red[NS * 2 * NLM * C];
  __shared__ float gg[2 * NLM * C];   // dJ/dGamma and dJ/dGamma_dot
  const int n = threadIdx.x % C, slot = threadIdx.x / C;
  const int nc = a.c0 + n;   // channel in the arrays
  const int64_t a0 = a.rr.chunk_rows[a.rr.chunk], a1 = a.rr.chunk_rows[a.rr.chunk + 1];
  const int64_t e0 = a.rr.row_ptr[a0];
  for (int64_t i = a0 + blockIdx.x; i < a1; i += gridDim.x) {
    const int64_t eb = a.rr.row_ptr[i], ee = a.rr.row_ptr[i + 1];
    float G[NLM], Gd[NLM], GG[NLM], GGd[NLM], ga[NP];
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      G[q] = a.gamma[(i * NLM + q) * CS + nc];
      Gd[q] = a.gammad[(i * NLM + q) * CS + nc];
      GG[q] = 0.0f;
      GGd[q] = 0.0f;
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) ga[q] = 0.0f;
    for (int64_t e = eb + slot; e < ee; e += NS) {
      const int64_t t = e - e0, ts = a.stack + t;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
      const float* Yd = a.geo2 + t * GEO_STRIDE + GEO_Y;
      float V[NCI], Vd[NCI], GV[NCI], GVd[NCI];
      load_V2<LMAX, NL, L, CS>(a, t, nc, Y, Yd, V, Vd);
#pragma unroll
      for (int q = 0; q < NCI; ++q) { GV[q] = 0.0f; GVd[q] = 0.0f; }
      static_for<0, NP>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr PathT pt = LP.p[k];
        constexpr int d3 = 2 * pt.l3 + 1;
        constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
        float GT[d3], GTd[d3];
#pragma unroll
        for (int m3 = 0; m3 < d3; ++m3) { GT[m3] = 0.0f; GTd[m3] = 0.0f; }
        if constexpr (pt.s_idx >= 0) {
          GT[0] = a.gs[(t * LP.n0e + pt.s_idx) * CS + nc];
          GTd[0] = a.gs[(ts * LP.n0e + pt.s_idx) * CS + nc];
        }
        if constexpr (pt.out_off >= 0) {
          const float al = a.alpha[k * CS + nc];
          float T[d3], Td[d3];
          path2<LMAX, NL, L, k>(V, Vd, G, Gd, T, Td);
          float gal = 0.0f;
#pragma unroll
          for (int m3 = 0; m3 < d3; ++m3) {
            const float gvo = a.gvout[(t * LP.n_out_comps + pt.out_off + m3) * CS + nc];
            const float gvod = a.gvout[(ts * LP.n_out_comps + pt.out_off + m3) * CS + nc];
            gal += gvo * T[m3] + gvod * Td[m3];
            GT[m3] += al * gvo;
            GTd[m3] += al * gvod;
          }
          ga[k] += gal;
        }
        // adjoints of T = C (V x G) and Td = C (Vd x G + V x Gd)
        static_for<0, nz.n>([&](auto Q) {
          constexpr int q = decltype(Q)::value;
          constexpr int i1 = pt.in_off + nz.m1[q], i2 = pt.l2 * pt.l2 + nz.m2[q], i3 = nz.m3[q];
          const float cgt = nz.c[q] * GT[i3], cgd = nz.c[q] * GTd[i3];
          GV[i1] += cgt * G[i2] + cgd * Gd[i2];
          GVd[i1] += cgd * G[i2];
          GG[i2] += cgt * V[i1] + cgd * Vd[i1];
          GGd[i2] += cgd * V[i1];
        });
      });
      if constexpr (L > 1) {
#pragma unroll
        for (int q = 0; q < NCI; ++q) {
          a.gvin[(t * NCI + q) * CS + nc] = GV[q];
          a.gvin[(ts * NCI + q) * CS + nc] = GVd[q];
        }
      } else {
        // V^0 = omega (x) Y, V^0_dot = omega_dot (x) Y + omega (x) Y_dot
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
          float go = 0.0f, god = 0.0f;
#pragma unroll
          for (int m = 0; m < 2 * l + 1; ++m) {
            go += GV[l * l + m] * Y[l * l + m] + GVd[l * l + m] * Yd[l * l + m];
            god += GVd[l * l + m] * Y[l * l + m];
          }
          a.gomega[(t * (LMAX + 1) + l) * CS + nc] = go;
          a.gomega[(ts * (LMAX + 1) + l) * CS + nc] = god;
        }
        if (a.badj) {
          // dJ/dY += GV omega + GVd omega_dot;  dJ/dY_dot += GVd omega
          float yb[9] = {}, ydb[9] = {};
#pragma unroll
          for (int l = 0; l <= LMAX; ++l) {
            const float w = a.omega1[(t * (LMAX + 1) + l) * CS + nc];
            const float wd = a.omega1[(ts * (LMAX + 1) + l) * CS + nc];
#pragma unroll
            for (int m = 0; m < 2 * l + 1; ++m) {
              yb[l * l + m] = GV[l * l + m] * w + GVd[l * l + m] * wd;
              ydb[l * l + m] = GVd[l * l + m] * w;
            }
          }
          add_ybar<C>(a.badj, t, ts, n, yb, ydb);
        }
      }
    }
    // dJ/dGamma and dJ/dGamma_dot summed over the slots, scaled by nbar^-1/2
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      red[(slot * 2 * NLM + q) * C + n] = GG[q];
      red[(slot * 2 * NLM + NLM + q) * C + n] = GGd[q];
    }
    __syncthreads();
    for (int q = slot; q < 2 * NLM; q += NS) {
      float v = 0.0f;
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) v += red[(s2 * 2 * NLM + q) * C + n];
      gg[q * C + n] = v * a.inv_sqrt_nbar;
    }
    __syncthreads();
    // alpha-gradient shares of this atom
    if constexpr (L < NL) {
      static_for<0, NP>([&](auto K) {
        constexpr int k = decltype(K)::value;
        red[slot * C + n] = ga[k];
        __syncthreads();
        if (slot == 0) {
          float v = 0.0f;
#pragma unroll
          for (int s = 0; s < NS; ++s) v += red[s * C + n];
          a.galpha[(i * NP + k) * CS + nc] = v;
        }
        __syncthreads();
      });
    }
    // Gamma = sum omega (x) Y;  Gamma_dot = sum omega_dot (x) Y + omega (x) Y_dot
    for (int64_t e = eb + slot; e < ee; e += NS) {
      const int64_t t = e - e0, ts = a.stack + t;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
      const float* Yd = a.geo2 + t * GEO_STRIDE + GEO_Y;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        float go = 0.0f, god = 0.0f;
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) {
          const float G = gg[(l * l + m) * C + n], Gd = gg[(NLM + l * l + m) * C + n];
          go += G * Y[l * l + m] + Gd * Yd[l * l + m];
          god += Gd * Y[l * l + m];
        }
        float* p0 = a.gomega + (t * (LMAX + 1) + l) * CS + nc;
        float* p1 = a.gomega + (ts * (LMAX + 1) + l) * CS + nc;
        if constexpr (L == 1) { *p0 += go; *p1 += god; } else { *p0 = go; *p1 = god; }
      }
      if (a.badj) {
        // dJ/dY += dJ/dGamma omega + dJ/dGamma_dot omega_dot;
        // dJ/dY_dot += dJ/dGamma_dot omega  (the sums carry nbar^-1/2)
        float yb[9] = {}, ydb[9] = {};
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
          const float w = a.omega[(t * (LMAX + 1) + l) * CS + nc];
          const float wd = a.omega[(ts * (LMAX + 1) + l) * CS + nc];
#pragma unroll
          for (int m = 0; m < 2 * l + 1; ++m) {
            const float G = gg[(l * l + m) * C + n], Gd = gg[(NLM + l * l + m) * C + n];
            yb[l * l + m] = G * w + Gd * wd;
            ydb[l * l + m] = Gd * w;
          }
        }
        add_ybar<C>(a.badj, t, ts, n, yb, ydb);
      }
    }
    __syncthreads();
  }
}

typedef void (*tp2_kernel_t)(TP2Args);

template <int LMAX, int NL, int C, int CS>
static tp2_kernel_t pick2(int L, bool bwd) {
  if (L == 1) return bwd ? k_tp2_bwd<LMAX, NL, 1, C, CS> : k_tp2_fwd<LMAX, NL, 1, C, CS>;
  if constexpr (NL >= 2) if (L == 2) return bwd ? k_tp2_bwd<LMAX, NL, 2, C, CS> : k_tp2_fwd<LMAX, NL, 2, C, CS>;
  if constexpr (NL >= 3) if (L == 3) return bwd ? k_tp2_bwd<LMAX, NL, 3, C, CS> : k_tp2_fwd<LMAX, NL, 3, C, CS>;
  return nullptr;
}

static tp2_kernel_t pick_tp2(int lmax, int NL, int L, int C, bool bwd) {
#define AFM_TP2(LM, NLV, CV) \
  if (lmax == LM && NL == NLV && C == CV) return pick2<LM, NLV, (CV > 64 ? 64 : CV), CV>(L, bwd);
  AFM_TP2(1, 1, 8)
  AFM_TP2(2, 1, 8)
  AFM_TP2(2, 2, 8)
  AFM_TP2(2, 2, 16)
  AFM_TP2(2, 2, 32)
  AFM_TP2(2, 2, 64)
  AFM_TP2(2, 3, 64)
  AFM_TP2(2, 2, 128)
#undef AFM_TP2
  return nullptr;
}

// one workgroup per atom; 128 channels run as two consecutive launches over
// the channel groups (the products are channelwise; the per-edge basis
// adjoints add group after group in a fixed order)
static int launch_tp2(tp2_kernel_t k, int C, TP2Args a, int64_t n_atoms, hipStream_t st) {
  const int CK = C > 64 ? 64 : C;
  for (int c0 = 0; c0 < C; c0 += CK) {
    a.c0 = c0;
    hipLaunchKernelGGL(k, dim3(grid_for(n_atoms, 1, 65536)), dim3(256), 0, st, a);
  }
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

// ----------------------------------------------------------------------------
// loaders / epilogues

struct LdAct {   // primal rows: silu(a); tangent rows: silu'(a) a_dot
  const float* pre; int ld; int stack;
  __device__ float operator()(int m, int k) const {
    if (m < stack) return silu_f(pre[(int64_t)m * ld + k]);
    const float a = pre[(int64_t)(m - stack) * ld + k];
    return d1silu(a) * pre[(int64_t)m * ld + k];
  }
  __device__ void load8(int m, int k, float* v) const {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (*this)(m, k + q);
  }
};
struct LdPlain {
  const float* x; int ld;
  __device__ float operator()(int m, int k) const { return x[(int64_t)m * ld + k]; }
  __device__ void load8(int m, int k, float* v) const {
    const float* p = x + (int64_t)m * ld + k;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = p[q];
  }
};
struct LdCat {
  const float* x; int w; const float* s; int ls;
  __device__ float operator()(int m, int k) const {
    return k < w ? x[(int64_t)m * w + k] : s[(int64_t)m * ls + (k - w)];
  }
  // values k .. k + 7 (all in range): one branch per group when the group
  // lies in one part
  __device__ void load8(int m, int k, float* v) const {
    if (k + 8 <= w) {
      const float* p = x + (int64_t)m * w + k;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[q];
    } else if (k >= w) {
      const float* p = s + (int64_t)m * ls + (k - w);
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[q];
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (*this)(m, k + q);
    }
  }
};
struct LdCoef {
  const float* c;
  __device__ float operator()(int m, int) const { return c[m]; }
};
// first two-body layer inputs: [onehot Zi | onehot Zj | rho] (primal rows)
// and [0 | 0 | rho_dot] (tangent rows)
struct LdZ {
  const float* geo; const float* geo2; const int32_t* eidx; const int32_t* col; const int32_t* species;
  int64_t e0_unused; RowRange rr; int stack, S, nb, p; float r_cut;
  __device__ float operator()(int m, int k) const {
    const int t = m < stack ? m : m - stack;
    const bool tan = m >= stack;
    if (k < 2 * S) {
      if (tan) return 0.0f;
      int64_t e0, e1;
      rr.get(e0, e1);
      const int z = k < S ? species[eidx[t]] : species[col[e0 + t]];
      return (min(max(z, 0), S - 1) == (k < S ? k : k - S)) ? 1.0f : 0.0f;
    }
    float rho, rhod;
    rho_pair(geo + (int64_t)t * GEO_STRIDE, geo2 + (int64_t)t * GEO_STRIDE, r_cut, p, k - 2 * S, rho, rhod);
    return tan ? rhod : rho;
  }
};
struct EpSt {
  float* y; int ld;
  __device__ void operator()(int m, int n, float v) const { y[(int64_t)m * ld + n] = v; }
};
struct EpAd {
  float* y; int ld;
  __device__ void operator()(int m, int n, float v) const { y[(int64_t)m * ld + n] += v; }
};
struct EpSplit2 {
  float* gx; int w; float* gs; int ls;
  __device__ void operator()(int m, int n, float v) const {
    if (n < w) gx[(int64_t)m * w + n] += v; else gs[(int64_t)m * ls + (n - w)] = v;
  }
};

// gacc[off + map(n, k)] += sum over slices (fixed order); env matrices map
// their l-major rows back to the layout's channel-major rows
__global__ void k_reduce_slices(const float* __restrict__ P, int slices, int N, int K, double* __restrict__ gacc,
                                int64_t off, int env_c, int env_l1) {
  const int64_t tot = (int64_t)N * K;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int s = 0; s < slices; ++s) v += (double)P[(int64_t)s * tot + q];
    int64_t n = q / K, k = q % K;
    if (env_c > 0) n = (n % env_c) * env_l1 + n / env_c;
    gacc[off + n * K + k] += v;
  }
}

// per-atom shares -> gacc (fixed order over atoms): a block owns 64
// columns; its 16 row groups sum atoms g, g + 16, ... and are combined in
// a fixed order
__global__ void __launch_bounds__(1024) k_reduce_atoms(const float* __restrict__ part, int64_t N, int64_t width,
                                                       double* __restrict__ gacc, int64_t off) {
  __shared__ double red[16][64];
  const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 64 + c;
  double v = 0.0;
  if (q < width)
    for (int64_t i = grp; i < N; i += 16) v += (double)part[i * width + q];
  red[grp][c] = v;
  __syncthreads();
  if (grp == 0 && q < width) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[k][c];
    gacc[off + q] += t;
  }
}

// one block per species: threads sum atoms tid, tid + 256, ... of that
// species, combined by a fixed-order tree
__global__ void __launch_bounds__(256) k_species_grad(const double* __restrict__ a_sig,
                                                      const double* __restrict__ a_mu,
                                                      const int32_t* __restrict__ species, int64_t N, int S,
                                                      double* __restrict__ gacc, int64_t off_sig, int64_t off_mu) {
  __shared__ double r1[256], r2[256];
  const int z = blockIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256)
    if (species[i] == z) { s1 += a_sig[i]; s2 += a_mu[i]; }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      r1[threadIdx.x] += r1[threadIdx.x + o];
      r2[threadIdx.x] += r2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    gacc[off_sig + z] += r1[0];
    gacc[off_mu + z] += r2[0];
  }
}

// dJ/dW_E1[h][f] = W_E2[h] q[f];  dJ/dW_E2[h] = sum_f W_E1[h][f] q[f]
__global__ void k_edge_grad(const double* __restrict__ q, const float* __restrict__ e0, const float* __restrict__ e1,
                            int H, int W, double* __restrict__ gacc, int64_t off0, int64_t off1) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)H * W + H;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx < (int64_t)H * W) {
      const int64_t h = idx / W, f = idx % W;
      gacc[off0 + idx] += (double)e1[h] * q[f];
    } else {
      const int64_t h = idx - (int64_t)H * W;
      double v = 0.0;
      for (int f = 0; f < W; ++f) v += (double)e0[h * W + f] * q[f];
      gacc[off1 + h] += v;
    }
  }
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    b[q] = (float)a[q];
}

// ----------------------------------------------------------------------------
// schedule

static int64_t block_offset(const afm_model* m, const char* name) {
  for (auto& b : m->blocks)
    if (strcmp(b.name, name) == 0) return b.offset;
  return -1;
}

template <class ALA, class ALB>
static int wgrad(bool bf16, hipStream_t st, RowRange rr, int stack, int N, int K, ALA A, ALB Bl, float* partial,
                 double* gacc, int64_t off, int env_c = 0, int env_l1 = 0) {
  const int rows = 2 * stack;
  const int tiles = ((N + 63) / 64) * ((K + 63) / 64);
  int slices = (4096 + tiles - 1) / tiles;   // ~16 workgroups per CU (1024: 14 % slower at 512 x 512)
  slices = slices < 1 ? 1 : (slices > kMaxSlices ? kMaxSlices : slices);
  const int rps = ((rows + slices - 1) / slices + 15) / 16 * 16;
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((K + 63) / 64), (unsigned)slices);
  if (bf16)
    hipLaunchKernelGGL((k_wgrad_bf16<ALA, ALB>), grid, dim3(256), 0, st, rr, stack, N, K, rps, A, Bl, partial);
  else
    hipLaunchKernelGGL((k_wgrad_mfma<ALA, ALB>), grid, dim3(256), 0, st, rr, stack, N, K, rps, A, Bl, partial);
  hipLaunchKernelGGL(k_reduce_slices, dim3(grid_for((int64_t)N * K, 256, 4096)), dim3(256), 0, st,
                     (const float*)partial, slices, N, K, gacc, off, env_c, env_l1);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

int launch_geometry(const afm_model* m, const SysDev& s, const NlDev& nl, const afm_workspace* ws, const WsLayout& L,
                    RowRange rr, hipStream_t st);   // forward.hip

int run_second_order(const afm_model* m, const SysDev& s, const NlDev& nl, const afm_workspace* ws,
                     const WsLayout& L, const double* gE, const double* gF, const double* gW, float* grad_out,
                     double* grad_pos, hipStream_t st) {
  TraceScope tr(st, "second_order");
  const ModelDims& d = m->dims;
  const Plan& P = m->plan;
  const bool so_bf16 = m->prec == AFM_BF16_MFMA;   // BF16 models: BF16 MFMA GEMMs, FP32 accumulation
  if (d.dense && d.NL > 1) {   // refuse before launching anything
    set_error("second-order pass not built for dense mixing");
    return AFM_E_UNSUPPORTED;
  }
  for (int layer = 1; layer <= d.NL; ++layer)
    if (!pick_tp2(d.lmax, d.NL, layer, d.c, false) || !pick_tp2(d.lmax, d.NL, layer, d.c, true)) {
      set_error("second-order tensor-product kernel not built for this shape");
      return AFM_E_UNSUPPORTED;
    }
  const int stack = (int)L.cex;
  const int64_t E2 = 2 * (int64_t)stack;
  const int env = (d.lmax + 1) * d.c;
  double* gacc = ws_ptr<double>(ws, L.so_gacc);
  float* partial = ws_ptr<float>(ws, L.so_partial);
  float* geo = ws_ptr<float>(ws, L.geo);
  int32_t* eidx = ws_ptr<int32_t>(ws, L.eidx);
  float* geo2 = ws_ptr<float>(ws, L.so_geo2);
  float* gx = ws_ptr<float>(ws, L.so_gx);
  float* ga = ws_ptr<float>(ws, L.so_ga);
  float* gh = ws_ptr<float>(ws, L.so_gh);
  float* gs2 = ws_ptr<float>(ws, L.so_gs);
  float* gom = ws_ptr<float>(ws, L.so_gomega);
  float* eps2 = ws_ptr<float>(ws, L.so_eps);
  float* coef = ws_ptr<float>(ws, L.so_coef);
  float* badj = grad_pos ? ws_ptr<float>(ws, L.so_badj) : nullptr;
  float* gpos_e = ws_ptr<float>(ws, L.so_gpos);
  int rc = zero_async(gacc, m->n_params * 8, st);
  if (!rc && grad_pos) rc = zero_async(gpos_e, nl.capacity * 12, st);
  if (!rc) rc = zero_async(ws_ptr<double>(ws, L.so_q), (int64_t)d.w * 8, st);
  if (rc) return rc;
  rc = launch_chunk_rows(s, nl, ws, L, st);
  if (!rc) rc = check_chunks(s, nl, ws, L, st);
  if (rc) return rc;
  RowRange rr{ws_ptr<int64_t>(ws, L.chunk_rows), nl.row_ptr, 0};
  const float inb = (float)(1.0 / sqrt(d.nbar));
  // activated stacked rows of a pre-activation buffer into gh (free wherever
  // a GEMM reads them; it holds at least w columns); false if F > w, where
  // the GEMM applies the activation in its loader instead
  auto act_into_gh = [&](const float* pre, int F) {
    if (F > d.w) return false;
    hipLaunchKernelGGL(k_act2_fwd, dim3(grid_for((int64_t)stack * F, 256, 65536)), dim3(256), 0, st, rr, stack, F,
                       pre, gh);
    return true;
  };
  for (int chunk = 0; chunk < ws->n_chunks; ++chunk) {
    rr.chunk = chunk;
    if (badj) {
      rc = zero_async(badj, E2 * kBadj * 4, st);
      if (rc) return rc;
    }
    // ---- forward with tangents ----
    rc = launch_geometry(m, s, nl, ws, L, rr, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_geom2, dim3(grid_for(stack, 256, 65536)), dim3(256), 0, st, rr, (const float*)geo,
                       (const int32_t*)eidx, (const int32_t*)nl.col, gF, gW, s.seg, s.B, (float)d.r_cut, d.p,
                       geo2);
    float* tbp0 = ws_ptr<float>(ws, L.so_tb_pre[0]);
    hipLaunchKernelGGL(k_tb2_first, dim3(grid_for((int64_t)stack * d.tb[0], 256, 65536)), dim3(256), 0, st, rr, stack,
                       (const float*)geo, (const float*)geo2, (const int32_t*)eidx, (const int32_t*)nl.col, s.species,
                       m->W.tb[0], d.S, d.nb, d.tb[0], (float)d.r_cut, d.p, tbp0);
    AFM_LAUNCH_CHECK();
    for (int k = 1; k < d.ntb; ++k) {
      const float* pa = ws_ptr<float>(ws, L.so_tb_pre[k - 1]);
      const EpSt ep{ws_ptr<float>(ws, L.so_tb_pre[k]), d.tb[k]};
      if (act_into_gh(pa, d.tb[k - 1]))
        sgemm_so<true>(so_bf16, st, rr, E2, d.tb[k - 1], d.tb[k], m->W.tb[k], d.tb[k - 1], LdPlain{gh, d.tb[k - 1]},
                       ep, stack);
      else
        sgemm_so<true>(so_bf16, st, rr, E2, d.tb[k - 1], d.tb[k], m->W.tb[k], d.tb[k - 1],
                       LdAct{pa, d.tb[k - 1], stack}, ep, stack);
    }
    float* x0 = ws_ptr<float>(ws, L.so_x[0]);
    hipLaunchKernelGGL(k_tb2_out, dim3(grid_for((int64_t)stack * d.w, 256, 65536)), dim3(256), 0, st, rr, stack, d.w,
                       (const float*)ws_ptr<float>(ws, L.so_tb_pre[d.ntb - 1]), (const float*)geo,
                       (const float*)geo2, x0);
    sgemm_so<true>(so_bf16, st, rr, E2, d.w, env, m->W.env[0], d.w, LdPlain{x0, d.w}, EpSt{ws_ptr<float>(ws, L.so_omega[0]), env},
                stack);
    AFM_LAUNCH_CHECK();
    for (int layer = 1; layer <= d.NL; ++layer) {
      const LayerPlan& lp = P.layer[layer - 1];
      const int ls = lp.n0e * d.c;
      TP2Args ta{};
      ta.rr = rr; ta.stack = stack; ta.geo = geo; ta.geo2 = geo2;
      ta.omega = ws_ptr<float>(ws, L.so_omega[layer - 1]);
      ta.omega1 = ws_ptr<float>(ws, L.so_omega[0]);
      ta.vin = layer > 1 ? ws_ptr<float>(ws, L.so_v[layer - 2]) : nullptr;
      ta.vout = layer < d.NL ? ws_ptr<float>(ws, L.so_v[layer - 1]) : nullptr;
      ta.s = ws_ptr<float>(ws, L.so_s[layer - 1]);
      ta.gamma = ws_ptr<float>(ws, L.gamma[layer - 1]);
      ta.gammad = ws_ptr<float>(ws, L.so_gammad[layer - 1]);
      ta.alpha = layer < d.NL ? m->W.alpha[layer - 1] : nullptr;
      ta.inv_sqrt_nbar = inb;
      tp2_kernel_t kf = pick_tp2(d.lmax, d.NL, layer, d.c, false);
      if (!kf) { set_error("second-order tensor-product kernel not built for this shape"); return AFM_E_UNSUPPORTED; }
      rc = launch_tp2(kf, d.c, ta, s.N, st);
      if (rc) return rc;
      const float* xp = ws_ptr<float>(ws, L.so_x[layer - 1]);
      for (int k = 0; k < d.depth; ++k) {
        float* pre = ws_ptr<float>(ws, L.so_lat_pre[layer - 1][k]);
        if (k == 0) {
          // [x | s] into gh (it holds w + max n0e c columns), then a plain GEMM
          hipLaunchKernelGGL(k_cat2, dim3(grid_for((int64_t)stack * (d.w + ls), 256, 65536)), dim3(256), 0, st, rr,
                             stack, xp, d.w, (const float*)ta.s, ls, gh);
          sgemm_so<true>(so_bf16, st, rr, E2, d.w + ls, d.w, m->W.lat[layer - 1][0], d.w + ls, LdPlain{gh, d.w + ls},
                         EpSt{pre, d.w}, stack);
        }
        else {
          act_into_gh(ws_ptr<float>(ws, L.so_lat_pre[layer - 1][k - 1]), d.w);
          sgemm_so<true>(so_bf16, st, rr, E2, d.w, d.w, m->W.lat[layer - 1][k], d.w, LdPlain{gh, d.w}, EpSt{pre, d.w},
                         stack);
        }
      }
      float* xn = ws_ptr<float>(ws, L.so_x[layer]);
      hipLaunchKernelGGL(k_lat2_out, dim3(grid_for((int64_t)stack * d.w, 256, 65536)), dim3(256), 0, st, rr, stack,
                         d.w, (const float*)ws_ptr<float>(ws, L.so_lat_pre[layer - 1][d.depth - 1]), xp,
                         (const float*)geo, (const float*)geo2, xn);
      if (layer < d.NL)
        sgemm_so<true>(so_bf16, st, rr, E2, d.w, env, m->W.env[layer], d.w, LdPlain{xn, d.w},
                    EpSt{ws_ptr<float>(ws, L.so_omega[layer]), env}, stack);
      AFM_LAUNCH_CHECK();
    }
    // ---- energies and the first adjoints ----
    const float* xN = ws_ptr<float>(ws, L.so_x[d.NL]);
    hipLaunchKernelGGL(k_energy2, dim3(grid_for(stack, 4, 16384)), dim3(256), 0, st, rr, stack, d.w, xN, m->W.w_eff,
                       (const int32_t*)eidx, s.species, m->W.sp_scale, d.S, d.escale, s.seg, s.B, gE, eps2, coef, gx);
    hipLaunchKernelGGL(k_atom2, dim3(grid_for(s.N, 256, 4096)), dim3(256), 0, st, rr, stack, (const float*)eps2,
                       s.species, d.S, d.escale, s.seg, s.B, gE, ws_ptr<double>(ws, L.so_asig),
                       ws_ptr<double>(ws, L.so_amu));
    AFM_LAUNCH_CHECK();
    // q[f] = sum_m coef_m x[m][f]  (accumulated in the q slot of gacc's tail)
    rc = wgrad(so_bf16, st, rr, stack, 1, d.w, LdCoef{coef}, LdPlain{xN, d.w}, partial, ws_ptr<double>(ws, L.so_q), 0);
    if (rc) return rc;
    // ---- reverse ----
    char nm[32];
    for (int layer = d.NL; layer >= 1; --layer) {
      const LayerPlan& lp = P.layer[layer - 1];
      const int ls = lp.n0e * d.c;
      const float* xp = ws_ptr<float>(ws, L.so_x[layer - 1]);
      if (layer < d.NL) {
        sgemm_so<false>(so_bf16, st, rr, E2, env, d.w, m->W.env[layer], d.w, LdPlain{gom, env}, EpAd{gx, d.w}, stack);
        snprintf(nm, sizeof nm, "layer%d.env", layer + 1);
        rc = wgrad(so_bf16, st, rr, stack, env, d.w, LdPlain{gom, env}, LdPlain{ws_ptr<float>(ws, L.so_x[layer]), d.w},
                   partial, gacc, block_offset(m, nm), d.c, d.lmax + 1);
        if (rc) return rc;
      }
      if (badj)
        hipLaunchKernelGGL(k_u2_adj, dim3(grid_for(stack, 4, 16384)), dim3(256), 0, st, rr, stack, d.w,
                           (const float*)ws_ptr<float>(ws, L.so_lat_pre[layer - 1][d.depth - 1]), (const float*)gx,
                           0.70710678118654752f, badj);
      hipLaunchKernelGGL(k_act2_bwd, dim3(grid_for((int64_t)stack * d.w, 256, 65536)), dim3(256), 0, st, rr, stack,
                         d.w, (const float*)ws_ptr<float>(ws, L.so_lat_pre[layer - 1][d.depth - 1]), gx, ga,
                         (const float*)geo, (const float*)geo2, 1, 0.70710678118654752f, 0.70710678118654752f);
      AFM_LAUNCH_CHECK();
      for (int k = d.depth - 1; k >= 0; --k) {
        snprintf(nm, sizeof nm, "layer%d.latent.%d", layer, k);
        const int64_t off = block_offset(m, nm);
        if (k > 0) {
          act_into_gh(ws_ptr<float>(ws, L.so_lat_pre[layer - 1][k - 1]), d.w);
          rc = wgrad(so_bf16, st, rr, stack, d.w, d.w, LdPlain{ga, d.w}, LdPlain{gh, d.w}, partial, gacc, off);
          if (rc) return rc;
          sgemm_so<false>(so_bf16, st, rr, E2, d.w, d.w, m->W.lat[layer - 1][k], d.w, LdPlain{ga, d.w}, EpSt{gh, d.w}, stack);
          hipLaunchKernelGGL(k_act2_bwd, dim3(grid_for((int64_t)stack * d.w, 256, 65536)), dim3(256), 0, st, rr,
                             stack, d.w, (const float*)ws_ptr<float>(ws, L.so_lat_pre[layer - 1][k - 1]), gh, ga,
                             (const float*)geo, (const float*)geo2, 0, 1.0f, 0.0f);
          AFM_LAUNCH_CHECK();
        } else {
          rc = wgrad(so_bf16, st, rr, stack, d.w, d.w + ls, LdPlain{ga, d.w},
                     LdCat{xp, d.w, ws_ptr<float>(ws, L.so_s[layer - 1]), ls}, partial, gacc, off);
          if (rc) return rc;
          sgemm_so<false>(so_bf16, st, rr, E2, d.w, d.w + ls, m->W.lat[layer - 1][0], d.w + ls, LdPlain{ga, d.w},
                       EpSplit2{gx, d.w, gs2, ls}, stack);
          AFM_LAUNCH_CHECK();
        }
      }
      TP2Args ta{};
      ta.rr = rr; ta.stack = stack; ta.geo = geo; ta.geo2 = geo2;
      ta.omega = ws_ptr<float>(ws, L.so_omega[layer - 1]);
      ta.omega1 = ws_ptr<float>(ws, L.so_omega[0]);
      ta.vin = layer > 1 ? ws_ptr<float>(ws, L.so_v[layer - 2]) : nullptr;
      ta.gamma = ws_ptr<float>(ws, L.gamma[layer - 1]);
      ta.gammad = ws_ptr<float>(ws, L.so_gammad[layer - 1]);
      ta.alpha = layer < d.NL ? m->W.alpha[layer - 1] : nullptr;
      ta.inv_sqrt_nbar = inb;
      ta.gs = gs2;
      float* gva = ws_ptr<float>(ws, L.so_gv0);
      float* gvb = ws_ptr<float>(ws, L.so_gv1);
      ta.gvout = (layer < d.NL) ? (((d.NL - layer) % 2 == 1) ? gva : gvb) : nullptr;
      ta.gvin = (layer > 1) ? (((d.NL - layer) % 2 == 0) ? gva : gvb) : nullptr;
      ta.gomega = gom;
      ta.galpha = layer < d.NL ? ws_ptr<float>(ws, L.so_galpha[layer - 1]) : nullptr;
      ta.badj = badj;
      tp2_kernel_t kb = pick_tp2(d.lmax, d.NL, layer, d.c, true);
      if (!kb) { set_error("second-order tensor-product kernel not built for this shape"); return AFM_E_UNSUPPORTED; }
      rc = launch_tp2(kb, d.c, ta, s.N, st);
      if (rc) return rc;
      // alpha shares are per atom (chunks do not overlap): reduced after the last chunk
    }
    // two-body reverse
    sgemm_so<false>(so_bf16, st, rr, E2, env, d.w, m->W.env[0], d.w, LdPlain{gom, env}, EpAd{gx, d.w}, stack);
    rc = wgrad(so_bf16, st, rr, stack, env, d.w, LdPlain{gom, env}, LdPlain{x0, d.w}, partial, gacc,
               block_offset(m, "layer1.env"), d.c, d.lmax + 1);
    if (rc) return rc;
    {
      const int F = d.tb[d.ntb - 1];
      if (badj)
        hipLaunchKernelGGL(k_u2_adj, dim3(grid_for(stack, 4, 16384)), dim3(256), 0, st, rr, stack, F,
                           (const float*)ws_ptr<float>(ws, L.so_tb_pre[d.ntb - 1]), (const float*)gx, 1.0f, badj);
      hipLaunchKernelGGL(k_act2_bwd, dim3(grid_for((int64_t)stack * F, 256, 65536)), dim3(256), 0, st, rr, stack, F,
                         (const float*)ws_ptr<float>(ws, L.so_tb_pre[d.ntb - 1]), gx, ga, (const float*)geo,
                         (const float*)geo2, 1, 1.0f, 0.0f);
      AFM_LAUNCH_CHECK();
      for (int k = d.ntb - 1; k >= 0; --k) {
        snprintf(nm, sizeof nm, "twobody.%d", k);
        const int64_t off = block_offset(m, nm);
        if (k > 0) {
          const float* pa = ws_ptr<float>(ws, L.so_tb_pre[k - 1]);
          if (act_into_gh(pa, d.tb[k - 1]))
            rc = wgrad(so_bf16, st, rr, stack, d.tb[k], d.tb[k - 1], LdPlain{ga, d.tb[k]}, LdPlain{gh, d.tb[k - 1]},
                       partial, gacc, off);
          else
            rc = wgrad(so_bf16, st, rr, stack, d.tb[k], d.tb[k - 1], LdPlain{ga, d.tb[k]},
                       LdAct{pa, d.tb[k - 1], stack}, partial, gacc, off);
          if (rc) return rc;
          sgemm_so<false>(so_bf16, st, rr, E2, d.tb[k], d.tb[k - 1], m->W.tb[k], d.tb[k - 1], LdPlain{ga, d.tb[k]},
                       EpSt{gh, d.tb[k - 1]}, stack);
          hipLaunchKernelGGL(k_act2_bwd, dim3(grid_for((int64_t)stack * d.tb[k - 1], 256, 65536)), dim3(256), 0, st,
                             rr, stack, d.tb[k - 1], (const float*)ws_ptr<float>(ws, L.so_tb_pre[k - 1]), gh, ga,
                             (const float*)geo, (const float*)geo2, 0, 1.0f, 0.0f);
          AFM_LAUNCH_CHECK();
        } else {
          LdZ lz{geo, geo2, eidx, nl.col, s.species, 0, rr, stack, d.S, d.nb, d.p, (float)d.r_cut};
          rc = wgrad(so_bf16, st, rr, stack, d.tb[0], 2 * d.S + d.nb, LdPlain{ga, d.tb[0]}, lz, partial, gacc, off);
          if (rc) return rc;
        }
      }
    }
    if (badj) {
      // basis adjoints complete for this chunk: rho from the first two-body
      // layer, then dJ/d delta per edge
      hipLaunchKernelGGL(k_rho2_adj, dim3(grid_for(2 * (int64_t)stack * d.nb, 256, 65536)), dim3(256), 0, st, rr,
                         stack, (const float*)ga, m->W.tb[0], d.S, d.nb, d.tb[0], badj);
      hipLaunchKernelGGL(k_gpos_edge, dim3(grid_for(stack, 256, 65536)), dim3(256), 0, st, rr, stack,
                         (const float*)geo, (const float*)geo2, (const float*)badj, (const int32_t*)eidx, gW, s.seg,
                         s.B, (float)d.r_cut, d.p, d.nb, gpos_e);
      AFM_LAUNCH_CHECK();
    }
  }
  if (grad_pos) {
    // dJ/dr_i = sum_{e in row i} (dJ/d delta_rev(e) - dJ/d delta_e)
    rc = run_edge_scatter(s, nl, gpos_e, grad_pos, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_negate_f64, dim3(grid_for(3 * s.N, 256, 4096)), dim3(256), 0, st, grad_pos, 3 * s.N);
    AFM_LAUNCH_CHECK();
  }
  // per-atom shares: alpha, species scale / shift; edge-energy matrices
  char nm[32];
  for (int layer = 1; layer < d.NL; ++layer) {
    snprintf(nm, sizeof nm, "layer%d.alpha", layer);
    const int64_t width = (int64_t)P.layer[layer - 1].n_paths * d.c;
    hipLaunchKernelGGL(k_reduce_atoms, dim3((unsigned)((width + 63) / 64)), dim3(1024), 0, st,
                       (const float*)ws_ptr<float>(ws, L.so_galpha[layer - 1]), s.N, width, gacc,
                       block_offset(m, nm));
  }
  hipLaunchKernelGGL(k_species_grad, dim3((unsigned)d.S), dim3(256), 0, st,
                     (const double*)ws_ptr<double>(ws, L.so_asig), (const double*)ws_ptr<double>(ws, L.so_amu),
                     s.species, s.N, d.S, gacc, block_offset(m, "species.scale"), block_offset(m, "species.shift"));
  hipLaunchKernelGGL(k_edge_grad, dim3(grid_for((int64_t)d.h * d.w + d.h, 256, 4096)), dim3(256), 0, st,
                     (const double*)ws_ptr<double>(ws, L.so_q), m->W.e0, m->W.e1, d.h, d.w, gacc,
                     block_offset(m, "edge.0"), block_offset(m, "edge.1"));
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(m->n_params, 256, 4096)), dim3(256), 0, st, (const double*)gacc,
                     grad_out, m->n_params);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

}  // namespace afm
