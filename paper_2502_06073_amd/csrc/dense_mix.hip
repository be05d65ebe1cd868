// Dense channel mixing after the tensor products: the alternative reading of
// the post-product mixing (Methodology / Model Training prints no equation),
// in which each path's outputs go through a c x c matrix,
//   V^L[ir3][n] = sum_{pi -> ir3} sum_k A^L_pi[n][k] T^pi[k]      (L < N_L),
// instead of one weight per (path, channel).  The matrices couple the
// channels, so an edge's tensor track is no longer a per-channel linear map
// of V^0 (the structure the per-path kernels are built on): here the
// per-edge features V^L, the products T^L and their adjoints are stored, the
// channelwise products and their adjoints run per atom (one group of C lanes
// per central atom, lane = channel), and the mixing is a GEMM over the edges
// of a chunk on the matrix cores (k_mix / k_mix_bwd in FP32 for FP32 models,
// k_mix_b16 / k_mix_b16_bwd on bf16 operand pairs for BF16 models), one per
// output component:
//   forward   V^L[t][ir3, m3][:] = A_ir3 [T^pi[t][m3][:] over pi -> ir3]
//   adjoint   dE/dT^pi[t][m3][:] = A_ir3^T dE/dV^L[t][ir3, m3][:]
// with A_ir3 = [A_pi1 | A_pi2 | ...] the path matrices side by side.
#include <hip/hip_runtime.h>

#include "cg_ct.h"
#include "device_util.h"
#include "gemm_f32.h"
#include "internal.h"

namespace afm {
namespace {

template <int LMAX, int NL, int L>
struct DenseCT {
  static constexpr LayerPlan lp = PlanCT<LMAX, NL>::plan.layer[L - 1];
};

template <bool B16>
__device__ __forceinline__ float ldx(const void* p, int64_t i) {
  if constexpr (B16) return __builtin_bit_cast(float, (uint32_t)static_cast<const uint16_t*>(p)[i] << 16);
  else return static_cast<const float*>(p)[i];
}
template <bool B16>
__device__ __forceinline__ void stx(void* p, int64_t i, float v) {
  if constexpr (B16) static_cast<uint16_t*>(p)[i] = __builtin_bit_cast(uint16_t, (__bf16)v);
  else static_cast<float*>(p)[i] = v;
}

// V^{L-1} of edge t, channel n: V^0 = omega^1 (x) Y for L = 1 (component
// l*l + m), else the stored features
template <int LMAX, int NL, int L, int C, bool B16>
__device__ __forceinline__ void load_vin(const DenseArgs& a, int64_t t, int n, const float* Y, float* V) {
  constexpr int NIN = DenseCT<LMAX, NL, L>::lp.n_in_comps;
  if constexpr (L == 1) {
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
      const float w = ldx<B16>(a.omega1, (t * (LMAX + 1) + l) * C + n);
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) V[l * l + m] = w * Y[l * l + m];
    }
  } else {
#pragma unroll
    for (int q = 0; q < NIN; ++q) V[q] = a.vin[(t * NIN + q) * C + n];
  }
}

// Forward of layer L: Gamma^L of each atom (stored for the adjoint), then per
// edge every path's product, the 0e outputs to s^L and, below the last
// layer, all products to the T buffer for the mixing GEMMs.
template <int LMAX, int NL, int L, int C, bool B16>
__global__ void __launch_bounds__(256) k_dtp_fwd(DenseArgs a) {
  constexpr LayerPlan LP = DenseCT<LMAX, NL, L>::lp;
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  constexpr int NIN = LP.n_in_comps, NT = dense_t_comps(LP), NS0 = LP.n0e;
  static_assert(L > 1 || NIN == NLM, "layer-1 inputs are omega^1 (x) Y");
  constexpr int NA = 256 / C;
  const int n = threadIdx.x % C, grp = threadIdx.x / C;
  const int64_t a0 = a.rr.chunk_rows[a.rr.chunk], a1 = a.rr.chunk_rows[a.rr.chunk + 1];
  const int64_t e0 = a.rr.row_ptr[a0];
  for (int64_t i = a0 + (int64_t)blockIdx.x * NA + grp; i < a1; i += (int64_t)gridDim.x * NA) {
    const int64_t eb = a.rr.row_ptr[i], ee = a.rr.row_ptr[i + 1];
    float G[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) G[q] = 0.0f;
    for (int64_t e = eb; e < ee; ++e) {
      const int64_t t = e - e0;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        const float w = ldx<B16>(a.omega, (t * (LMAX + 1) + l) * C + n);
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) G[l * l + m] += w * Y[l * l + m];
      }
    }
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      G[q] *= a.inv_sqrt_nbar;
      a.gamma[(i * NLM + q) * C + n] = G[q];
    }
    for (int64_t e = eb; e < ee; ++e) {
      const int64_t t = e - e0;
      float Y[NLM];
#pragma unroll
      for (int q = 0; q < NLM; ++q) Y[q] = a.geo[t * GEO_STRIDE + GEO_Y + q];
      float V[NIN];
      load_vin<LMAX, NL, L, C, B16>(a, t, n, Y, V);
      static_for<0, LP.n_paths>([&](auto P) {
        constexpr int k = decltype(P)::value;
        constexpr PathT pt = LP.p[k];
        static_assert(L > 1 || pt.in_off == pt.l1 * pt.l1, "layer-1 input offsets");
        constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
        float T[2 * pt.l3 + 1];
#pragma unroll
        for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) T[m3] = 0.0f;
        static_for<0, nz.n>([&](auto Q) {
          constexpr int q = decltype(Q)::value;
          T[nz.m3[q]] += nz.c[q] * V[pt.in_off + nz.m1[q]] * G[pt.l2 * pt.l2 + nz.m2[q]];
        });
        if constexpr (pt.s_idx >= 0) stx<B16>(a.s, (t * NS0 + pt.s_idx) * C + n, T[0]);
        if constexpr (L < NL && pt.out_off >= 0) {
          constexpr int to = dense_t_off(LP, k);
#pragma unroll
          for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) a.tbuf[(t * NT + to + m3) * C + n] = T[m3];
        }
      });
    }
  }
}

// Adjoint of layer L: dE/dT^pi = dE/ds (0e paths) + the mixing adjoint
// (T buffer, L < N_L); per edge dE/dV^{L-1} = sum C Gamma dE/dT (stored),
// per atom dE/dGamma = sum over the row of C V^{L-1} dE/dT; then per edge
// dE/domega^L (written) and the channel sums of dE/dY (added), with layer 1
// adding its inputs' adjoint dE/dV^0 through V^0 = omega^1 (x) Y.
template <int LMAX, int NL, int L, int C, bool B16>
__global__ void __launch_bounds__(256) k_dtp_bwd(DenseArgs a) {
  constexpr LayerPlan LP = DenseCT<LMAX, NL, L>::lp;
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  constexpr int NIN = LP.n_in_comps, NT = dense_t_comps(LP), NS0 = LP.n0e;
  static_assert(L > 1 || NIN == NLM, "layer-1 inputs are omega^1 (x) Y");
  constexpr int NA = 256 / C;
  const int n = threadIdx.x % C, grp = threadIdx.x / C;
  const int64_t a0 = a.rr.chunk_rows[a.rr.chunk], a1 = a.rr.chunk_rows[a.rr.chunk + 1];
  const int64_t e0 = a.rr.row_ptr[a0];
  for (int64_t i = a0 + (int64_t)blockIdx.x * NA + grp; i < a1; i += (int64_t)gridDim.x * NA) {
    const int64_t eb = a.rr.row_ptr[i], ee = a.rr.row_ptr[i + 1];
    float G[NLM], GG[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      G[q] = a.gamma[(i * NLM + q) * C + n];
      GG[q] = 0.0f;
    }
    for (int64_t e = eb; e < ee; ++e) {
      const int64_t t = e - e0;
      float Y[NLM];
#pragma unroll
      for (int q = 0; q < NLM; ++q) Y[q] = a.geo[t * GEO_STRIDE + GEO_Y + q];
      float V[NIN], dV[NIN];
      load_vin<LMAX, NL, L, C, B16>(a, t, n, Y, V);
#pragma unroll
      for (int q = 0; q < NIN; ++q) dV[q] = 0.0f;
      static_for<0, LP.n_paths>([&](auto P) {
        constexpr int k = decltype(P)::value;
        constexpr PathT pt = LP.p[k];
        constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
        float dT[2 * pt.l3 + 1];
#pragma unroll
        for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) dT[m3] = 0.0f;
        if constexpr (pt.s_idx >= 0) dT[0] = ldx<B16>(a.gs, (t * NS0 + pt.s_idx) * C + n);
        if constexpr (L < NL && pt.out_off >= 0) {
          constexpr int to = dense_t_off(LP, k);
#pragma unroll
          for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) dT[m3] += a.tbuf[(t * NT + to + m3) * C + n];
        }
        static_for<0, nz.n>([&](auto Q) {
          constexpr int q = decltype(Q)::value;
          const float cg = nz.c[q] * dT[nz.m3[q]];
          GG[pt.l2 * pt.l2 + nz.m2[q]] += cg * V[pt.in_off + nz.m1[q]];
          dV[pt.in_off + nz.m1[q]] += cg * G[pt.l2 * pt.l2 + nz.m2[q]];
        });
      });
      // L >= 2: input of the layer below's mixing adjoint; L = 1: dE/dV^0,
      // read back by the pass below
#pragma unroll
      for (int q = 0; q < NIN; ++q) a.dvbuf[(t * NIN + q) * C + n] = dV[q];
    }
#pragma unroll
    for (int q = 0; q < NLM; ++q) GG[q] *= a.inv_sqrt_nbar;
    for (int64_t e = eb; e < ee; ++e) {
      const int64_t t = e - e0;
      float tot[NLM];
#pragma unroll
      for (int q = 0; q < NLM; ++q) {
        tot[q] = GG[q];
        if constexpr (L == 1) tot[q] += a.dvbuf[(t * NLM + q) * C + n];
      }
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        const float w = ldx<B16>(a.omega, (t * (LMAX + 1) + l) * C + n);
        float go = 0.0f;
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) {
          const int q = l * l + m;
          go += tot[q] * a.geo[t * GEO_STRIDE + GEO_Y + q];
          const float y = group_sum<C>(tot[q] * w);
          if (n == 0) a.gy[t * GEO_STRIDE + q] += y;
        }
        stx<B16>(a.gomega, (t * (LMAX + 1) + l) * C + n, go);
      }
    }
  }
}

typedef void (*dense_kernel_t)(DenseArgs);

template <int LMAX, int NL, int C, bool B16>
dense_kernel_t pick_dense(int L, bool bwd) {
  if (L == 1) return bwd ? k_dtp_bwd<LMAX, NL, 1, C, B16> : k_dtp_fwd<LMAX, NL, 1, C, B16>;
  if constexpr (NL >= 2) if (L == 2) return bwd ? k_dtp_bwd<LMAX, NL, 2, C, B16> : k_dtp_fwd<LMAX, NL, 2, C, B16>;
  if constexpr (NL >= 3) if (L == 3) return bwd ? k_dtp_bwd<LMAX, NL, 3, C, B16> : k_dtp_fwd<LMAX, NL, 3, C, B16>;
  return nullptr;
}

template <int LMAX, int C, bool B16>
dense_kernel_t pick_dense_nl(int NL, int L, bool bwd) {
  switch (NL) {
    case 2: return pick_dense<LMAX, 2, C, B16>(L, bwd);
    case 3: return pick_dense<LMAX, 3, C, B16>(L, bwd);
  }
  return nullptr;
}

template <int LMAX, bool B16>
dense_kernel_t pick_dense_c(int C, int NL, int L, bool bwd) {
  switch (C) {
    case 8: return pick_dense_nl<LMAX, 8, B16>(NL, L, bwd);
    case 16: return pick_dense_nl<LMAX, 16, B16>(NL, L, bwd);
    case 32: return pick_dense_nl<LMAX, 32, B16>(NL, L, bwd);
    case 64: return pick_dense_nl<LMAX, 64, B16>(NL, L, bwd);
  }
  return nullptr;
}

template <bool B16>
dense_kernel_t pick_dense_l(int lmax, int C, int NL, int L, bool bwd) {
  switch (lmax) {
    case 0: return pick_dense_c<0, B16>(C, NL, L, bwd);
    case 1: return pick_dense_c<1, B16>(C, NL, L, bwd);
    case 2: return pick_dense_c<2, B16>(C, NL, L, bwd);
  }
  return nullptr;
}

// One mixing GEMM: output irrep r at component m3 over the chunk's edges.
// Forward  V[t][off][n] = sum_k T(t, k) W[n][k],  k = (path j, channel c),
//          T(t, k) = T[t][toff[j] + m3][c];
// adjoint  dT(t, k) = sum_n dV[t][off][n] W[n][k]   (W = A_r, [C][np C]).
struct MixOps {
  const float* x;    // forward: T buffer; adjoint: dE/dV
  float* y;          // forward: V^L; adjoint: dE/dT
  const float* W;    // A_r, row-major [C][np C]
  int C, np, nt, nv, off, m3;
  int toff[kMaxPaths];
};

// Forward GEMM: 64 edges x the C <= 64 output channels per workgroup (4
// wavefronts of 32 x 32 on v_mfma_f32_16x16x4f32: FP32 products and sums),
// the np C reduction staged 32 at a time through LDS with 16-byte loads; a
// reduction run of 4 never crosses a path (C is a multiple of 4), so every
// load is one aligned float4.
__global__ void __launch_bounds__(256) k_mix(RowRange rr, MixOps o) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int m0 = blockIdx.x * 64;
  if (m0 >= M) return;
  const int K = o.np * o.C, N = o.C;
  constexpr int KS = 32;
  __shared__ __attribute__((aligned(16))) float As[KS][68];   // [k][row]
  __shared__ __attribute__((aligned(16))) float Bs[KS][68];   // [k][column]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int lr = lane & 15, lk = lane >> 4;
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float4 ra[2], rb[2];
  // stage k0: T rows r = idx / 8 and W rows (output channels) r, reduction
  // k0 + 4 (idx % 8)
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx >> 3, k = k0 + 4 * (idx & 7);
      const int m = m0 + r;
      ra[q] = z4;
      if (m < M && k < K) {
        const int j = k / o.C;
        ra[q] = *reinterpret_cast<const float4*>(o.x + ((int64_t)m * o.nt + o.toff[j] + o.m3) * o.C + (k - j * o.C));
      }
      rb[q] = (r < N && k < K) ? *reinterpret_cast<const float4*>(o.W + (int64_t)r * K + k) : z4;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += KS) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx >> 3, kk = 4 * (idx & 7);
      As[kk + 0][r] = ra[q].x;
      As[kk + 1][r] = ra[q].y;
      As[kk + 2][r] = ra[q].z;
      As[kk + 3][r] = ra[q].w;
      Bs[kk + 0][r] = rb[q].x;
      Bs[kk + 1][r] = rb[q].y;
      Bs[kk + 2][r] = rb[q].z;
      Bs[kk + 3][r] = rb[q].w;
    }
    __syncthreads();
    if (k0 + KS < K) fetch(k0 + KS);
#pragma unroll
    for (int s4 = 0; s4 < KS / 4; ++s4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[4 * s4 + lk][32 * wr + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[4 * s4 + lk][32 * wc + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f32(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m0 + 32 * wr + 16 * i + 4 * lk + q;
      if (m >= M) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = 32 * wc + 16 * j + lr;
        if (n < N) o.y[((int64_t)m * o.nv + o.off) * o.C + n] = acc[i][j][q];
      }
    }
}

// Adjoint GEMM: the reduction runs over the C <= 64 output channels only,
// so a workgroup stages its 64 rows of dE/dV once ([k][row] in LDS) and
// sweeps up to kMixBwdTiles tiles of 64 of the np C output columns (all of
// them for every built model), the next W tile fetched into registers while
// the current one is multiplied (one tile per workgroup instead measured
// 1.4x slower: the rows were staged once per tile).
constexpr int kMixBwdTiles = 16;
__global__ void __launch_bounds__(256) k_mix_bwd(RowRange rr, MixOps o) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int m0 = blockIdx.x * 64;
  if (m0 >= M) return;
  const int K = o.C, N = o.np * o.C;
  const int nb = blockIdx.y * 64 * kMixBwdTiles, ne = nb + 64 * kMixBwdTiles < N ? nb + 64 * kMixBwdTiles : N;
  __shared__ __attribute__((aligned(16))) float As[64][68];   // [k][row]
  __shared__ __attribute__((aligned(16))) float Bs[64][68];   // [k][column]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // dE/dV rows: row r = idx / 16, channels 4 (idx % 16)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q;
    const int r = idx >> 4, k = 4 * (idx & 15);
    const int m = m0 + r;
    float4 v = z4;
    if (m < M && k < K) v = *reinterpret_cast<const float4*>(o.x + ((int64_t)m * o.nv + o.off) * o.C + k);
    As[k + 0][r] = v.x;
    As[k + 1][r] = v.y;
    As[k + 2][r] = v.z;
    As[k + 3][r] = v.w;
  }
  // W tile of columns [n0, n0 + 64): row k = idx / 16, columns 4 (idx % 16)
  float4 rb[4];
  auto fetch = [&](int n0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int k = idx >> 4, n = n0 + 4 * (idx & 15);
      rb[q] = (k < K && n < N) ? *reinterpret_cast<const float4*>(o.W + (int64_t)k * N + n) : z4;
    }
  };
  fetch(nb);
  for (int n0 = nb; n0 < ne; n0 += 64) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      *reinterpret_cast<float4*>(&Bs[idx >> 4][4 * (idx & 15)]) = rb[q];
    }
    __syncthreads();
    if (n0 + 64 < ne) fetch(n0 + 64);
    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    for (int s4 = 0; s4 < K / 4; ++s4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[4 * s4 + lk][32 * wr + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[4 * s4 + lk][32 * wc + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f32(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 32 * wr + 16 * i + 4 * lk + q;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int n = n0 + 32 * wc + 16 * j + lr;
          if (n >= N) continue;
          const int jp = n / o.C;
          o.y[((int64_t)m * o.nt + o.toff[jp] + o.m3) * o.C + (n - jp * o.C)] = acc[i][j][q];
        }
      }
  }
}

// BF16 models: the same GEMMs on v_mfma_f32_16x16x32_bf16 with both
// operands as bf16 pairs (x = x_hi + x_lo, w = w_hi + w_lo; the pairs of W
// made at model creation, those of the activations when a stage is staged)
// and three products per block, x_hi w_hi + x_hi w_lo + x_lo w_hi (the
// dropped x_lo w_lo is ~2^-16 of the product): FP32-like accuracy at a
// fraction of the FP32 matrix-core time.  Forward: 64 edges x the C <= 64
// output channels per workgroup, X = T (K = np C) staged 32 at a time,
// W rows = A_r ([C][K]).
__global__ void __launch_bounds__(256) k_mix_b16(RowRange rr, MixOps o, const __bf16* __restrict__ Wh,
                                                 const __bf16* __restrict__ Wl) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int m0 = blockIdx.x * 64;
  if (m0 >= M) return;
  const int n0 = 0;
  const int K = o.np * o.C, N = o.C;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[64 * kBfRow], Al[64 * kBfRow];   // [row][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bh[64 * kBfRow], Bl[64 * kBfRow];   // [column][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int lr = lane & 15, lg = lane >> 4;
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const uint4 zu = make_uint4(0u, 0u, 0u, 0u);
  // stage k0: X rows r = idx / 8, reduction k0 + 4 (idx % 8) (two float4 per
  // thread); W rows (output columns) n0 + tid / 4, k0 + 8 (tid % 4) (one run
  // of 8 bf16 per term)
  float4 ra[2];
  uint4 rh, rl;
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx >> 3, k = k0 + 4 * (idx & 7);
      const int m = m0 + r;
      ra[q] = z4;
      if (m < M && k < K) {
        const int j = k / o.C;
        ra[q] = *reinterpret_cast<const float4*>(o.x + ((int64_t)m * o.nt + o.toff[j] + o.m3) * o.C + (k - j * o.C));
      }
    }
    const int n = n0 + (tid >> 2), k = k0 + 8 * (tid & 3);
    rh = zu;
    rl = zu;
    if (n < N && k < K) {
      rh = *reinterpret_cast<const uint4*>(Wh + (int64_t)n * K + k);
      rl = *reinterpret_cast<const uint4*>(Wl + (int64_t)n * K + k);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += 32) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx >> 3, kk = 4 * (idx & 7);
      const float v[4] = {ra[q].x, ra[q].y, ra[q].z, ra[q].w};
      __bf16 h[4], l[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        h[c] = (__bf16)v[c];
        l[c] = (__bf16)(v[c] - (float)h[c]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Ah[r * kBfRow + kk + c] = h[c];
        Al[r * kBfRow + kk + c] = l[c];
      }
    }
    *reinterpret_cast<uint4*>(&Bh[(tid >> 2) * kBfRow + 8 * (tid & 3)]) = rh;
    *reinterpret_cast<uint4*>(&Bl[(tid >> 2) * kBfRow + 8 * (tid & 3)]) = rl;
    __syncthreads();
    if (k0 + 32 < K) fetch(k0 + 32);
    bf16x8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = lds_row8(Ah, 32 * wr + 16 * i + lr, lg);
      al[i] = lds_row8(Al, 32 * wr + 16 * i + lr, lg);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      bh[j] = lds_row8(Bh, 32 * wc + 16 * j + lr, lg);
      bl[j] = lds_row8(Bl, 32 * wc + 16 * j + lr, lg);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = mfma_bf16(ah[i], bh[j], acc[i][j]);
        acc[i][j] = mfma_bf16(ah[i], bl[j], acc[i][j]);
        acc[i][j] = mfma_bf16(al[i], bh[j], acc[i][j]);
      }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m0 + 32 * wr + 16 * i + 4 * lg + q;
      if (m >= M) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + 32 * wc + 16 * j + lr;
        if (n < N) o.y[((int64_t)m * o.nv + o.off) * o.C + n] = acc[i][j][q];
      }
    }
}

// Adjoint on bf16 pairs with the rows staged once: a workgroup splits its
// 64 rows of dE/dV (K = C <= 64) into LDS, then sweeps the np C output
// columns 64 at a time (W = A_r^T pairs, the next tile fetched into
// registers while the current one is multiplied; one column tile per
// workgroup, the rows staged once per tile, measured 1.2x slower).
constexpr int kRowK = 72;   // bf16 per LDS row: 64 reduction values + 8 of padding (16-byte aligned rows)
__device__ __forceinline__ bf16x8_t lds_row8k(const __bf16* T, int r, int k) {
  return *reinterpret_cast<const bf16x8_t*>(T + r * kRowK + k);
}
__global__ void __launch_bounds__(256) k_mix_b16_bwd(RowRange rr, MixOps o, const __bf16* __restrict__ Wh,
                                                     const __bf16* __restrict__ Wl) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int m0 = blockIdx.x * 64;
  if (m0 >= M) return;
  const int K = o.C, N = o.np * o.C;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[64 * kRowK], Al[64 * kRowK];   // [row][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bh[64 * kRowK], Bl[64 * kRowK];   // [column][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int lr = lane & 15, lg = lane >> 4;
  const uint4 zu = make_uint4(0u, 0u, 0u, 0u);
  // rows r = idx / 16, channels 4 (idx % 16)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + 256 * q;
    const int r = idx >> 4, k = 4 * (idx & 15);
    const int m = m0 + r;
    float4 x = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (m < M && k < K) x = *reinterpret_cast<const float4*>(o.x + ((int64_t)m * o.nv + o.off) * o.C + k);
    const float v[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const __bf16 h = (__bf16)v[c];
      Ah[r * kRowK + k + c] = h;
      Al[r * kRowK + k + c] = (__bf16)(v[c] - (float)h);
    }
  }
  // W tile: columns n0 + idx / 8, reduction 8 (idx % 8)
  uint4 rh[2], rl[2];
  auto fetch = [&](int n0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      const int n = n0 + (idx >> 3), k = 8 * (idx & 7);
      rh[q] = zu;
      rl[q] = zu;
      if (n < N && k < K) {
        rh[q] = *reinterpret_cast<const uint4*>(Wh + (int64_t)n * K + k);
        rl[q] = *reinterpret_cast<const uint4*>(Wl + (int64_t)n * K + k);
      }
    }
  };
  fetch(0);
  const int ks = (K + 31) / 32;
  for (int n0 = 0; n0 < N; n0 += 64) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      *reinterpret_cast<uint4*>(&Bh[(idx >> 3) * kRowK + 8 * (idx & 7)]) = rh[q];
      *reinterpret_cast<uint4*>(&Bl[(idx >> 3) * kRowK + 8 * (idx & 7)]) = rl[q];
    }
    __syncthreads();
    if (n0 + 64 < N) fetch(n0 + 64);
    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    for (int st = 0; st < ks; ++st) {
      const int kb = 32 * st + 8 * lg;
      bf16x8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ah[i] = lds_row8k(Ah, 32 * wr + 16 * i + lr, kb);
        al[i] = lds_row8k(Al, 32 * wr + 16 * i + lr, kb);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        bh[j] = lds_row8k(Bh, 32 * wc + 16 * j + lr, kb);
        bl[j] = lds_row8k(Bl, 32 * wc + 16 * j + lr, kb);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = mfma_bf16(ah[i], bh[j], acc[i][j]);
          acc[i][j] = mfma_bf16(ah[i], bl[j], acc[i][j]);
          acc[i][j] = mfma_bf16(al[i], bh[j], acc[i][j]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 32 * wr + 16 * i + 4 * lg + q;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int n = n0 + 32 * wc + 16 * j + lr;
          if (n >= N) continue;
          const int jp = n / o.C;
          o.y[((int64_t)m * o.nt + o.toff[jp] + o.m3) * o.C + (n - jp * o.C)] = acc[i][j][q];
        }
      }
  }
}

}  // namespace

int launch_dense_tp(int lmax, int NL, int L, int C, bool bwd, bool bf16, const DenseArgs& a,
                    int64_t n_atoms_max, hipStream_t st) {
  dense_kernel_t k = bf16 ? pick_dense_l<true>(lmax, C, NL, L, bwd) : pick_dense_l<false>(lmax, C, NL, L, bwd);
  if (!k) { set_error("dense-mixing tensor-product kernel not built for this shape"); return AFM_E_UNSUPPORTED; }
  hipLaunchKernelGGL(k, dim3(grid_for(n_atoms_max, 256 / C, 65536)), dim3(256), 0, st, a);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

// Mixing of layer L (< N_L) over the edges of a chunk (at most E rows).
// Forward: T (tbuf) -> V^L (feat).  Adjoint: dE/dV^L (feat) -> dE/dT (tbuf),
// every component of the paths with an output written.
int launch_dense_mix(const afm_model* m, int L, bool bwd, RowRange rr, int64_t E, float* feat, float* tbuf,
                     hipStream_t st) {
  const ModelDims& d = m->dims;
  const LayerPlan& lp = m->plan.layer[L - 1];
  const int nt = dense_t_comps(lp), nv = lp.n_out_comps;
  for (int r = 0; r < lp.n_out; ++r) {
    int toff[kMaxPaths] = {}, np = 0;
    for (int k = 0; k < lp.n_paths; ++k)
      if (lp.p[k].out_off == lp.out_off[r]) toff[np++] = dense_t_off(lp, k);
    if (np == 0) continue;
    MixOps o{};
    o.x = bwd ? feat : tbuf;
    o.y = bwd ? tbuf : feat;
    o.W = m->W.mix[L - 1] + m->W.mix_off[L - 1][r];
    o.C = d.c; o.np = np; o.nt = nt; o.nv = nv;
    for (int j = 0; j < np; ++j) o.toff[j] = toff[j];
    const unsigned gx = (unsigned)((E + 63) / 64 > 0 ? (E + 63) / 64 : 1);
    const int ntile = (np * d.c + 64 * kMixBwdTiles - 1) / (64 * kMixBwdTiles);
    const bool b16 = m->prec == AFM_BF16_MFMA;
    const int64_t T = m->W.mix_elems[L - 1], wo = m->W.mix_off[L - 1][r];
    const __bf16* wb = reinterpret_cast<const __bf16*>(m->W.mix_b16[L - 1]);
    if (b16 && !wb) { set_error("internal: bf16 mixing weights missing"); return AFM_E_INVALID; }
    for (int m3 = 0; m3 < 2 * lp.out[r].l + 1; ++m3) {
      o.m3 = m3;
      o.off = lp.out_off[r] + m3;
      if (b16 && bwd)
        hipLaunchKernelGGL(k_mix_b16_bwd, dim3(gx), dim3(256), 0, st, rr, o, wb + 2 * T + wo, wb + 3 * T + wo);
      else if (b16)
        hipLaunchKernelGGL(k_mix_b16, dim3(gx), dim3(256), 0, st, rr, o, wb + wo, wb + T + wo);
      else if (bwd)
        hipLaunchKernelGGL(k_mix_bwd, dim3(gx, (unsigned)ntile), dim3(256), 0, st, rr, o);
      else
        hipLaunchKernelGGL(k_mix, dim3(gx), dim3(256), 0, st, rr, o);
      AFM_LAUNCH_CHECK();
    }
  }
  return AFM_OK;
}

}  // namespace afm
