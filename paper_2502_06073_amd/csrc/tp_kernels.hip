// Environment sums and channelwise Clebsch-Gordan tensor products (the
// "tensor features ... l = 2 in full O(3)" of Methodology / Model Training).
//
// One workgroup per central atom i (all edges of row i): 256 threads =
// (256 / C) edge slots x C channels, channel fastest so every load is
// coalesced over channels.
//   forward:  Gamma_i[lm][n] = nbar^-1/2 sum_{e in row i} omega_e[l][n] Y_e[lm]
//             T^pi_e[m3][n] = sum C^{l1 l2 l3}[m1][m2][m3] V_e[l1 p1, m1][n] Gamma_i[l2 m2][n]
//             s_e (0e paths), V'_e = sum_pi alpha[pi][n] T^pi_e   (next layer)
//   backward: the adjoints of both lines; dE/dGamma_i is accumulated per
//             thread over the row's edges (9 registers) and reduced over the
//             edge slots in LDS.
// Per-edge tensor features never go to memory: V^{L-1} is rebuilt from
// V^0 = omega^1 (x) Y through the earlier layers' Gammas, and dE/dV^L from
// the later layers' dE/ds and Gammas, a few hundred FLOP per channel in
// place of 2-4 KB per edge written and read back.
// The sums run over the nonzero CG entries only, unrolled with immediate
// coefficients from the compile-time tables (cg_ct.h); Gamma_i of the
// thread's channel stays in registers for the whole row.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "gemm_f32.h"
#include "cg_ct.h"
#include "internal.h"

namespace afm {


__device__ __forceinline__ uint16_t to_bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
// element i of a float (B16 false) or bf16 (B16 true) array
template <bool B16>
__device__ __forceinline__ float ld_w(const void* p, int64_t i) {
  if constexpr (B16) return __builtin_bit_cast(float, (uint32_t)static_cast<const uint16_t*>(p)[i] << 16);
  else return static_cast<const float*>(p)[i];
}
template <bool B16>
__device__ __forceinline__ void st_w(void* p, int64_t i, float v) {
  if constexpr (B16) static_cast<uint16_t*>(p)[i] = to_bf16_bits(v);
  else static_cast<float*>(p)[i] = v;
}
// dst[q] += sum over the C channels (lanes n of one group) of v[q], q < NV
template <int C, int NV>
__device__ __forceinline__ void add_channel_sums(float (&v)[16], float* dst, int n) {
  if constexpr (C == 64) {
    const float y = wave_sum16(v, n);
    if ((n & 3) == 0 && (n >> 2) < NV) dst[n >> 2] += y;
  } else {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const float y = group_sum<C>(v[q]);
      if (n == 0) dst[q] += y;
    }
  }
}

template <int LMAX, int NL, int L>
struct LayerCT {
  static constexpr LayerPlan lp = PlanCT<LMAX, NL>::plan.layer[L - 1];
};

// Gamma of layers L0 + 1 .. L0 + NG of atom i, channel n (registers)
template <int LMAX, int L0, int NG, int C, int ND>
__device__ __forceinline__ void load_gammas(const TPArgs& a, int64_t i, int n,
                                            float (&Gs)[ND][(LMAX + 1) * (LMAX + 1)]) {
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  static_assert(NG <= ND, "gamma registers");
#pragma unroll
  for (int l = 0; l < NG; ++l)
#pragma unroll
    for (int q = 0; q < NLM; ++q) Gs[l][q] = a.gamma_l[L0 + l][(i * NLM + q) * C + n];
}

template <int LMAX, int NL, int L, int K>
__device__ __forceinline__ void path_fwd(const float* V, const float* G, float* T);

// Output features of layer K (V^K, the input of layer K + 1) for edge t,
// channel n, recomputed from V^0 = omega^1 (x) Y through layers 1..K with
// Gamma^l = Gp[l - 1] and the mixing weights alpha^l.
template <int LMAX, int NL, int K, int C, bool B16, int NG>
__device__ __forceinline__ void recompute_V(const TPArgs& a, int64_t t, int n, const float* Y,
                                            const float (&Gp)[NG][(LMAX + 1) * (LMAX + 1)], float* V) {
  if constexpr (K == 0) {
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
      const float w = ld_w<B16>(a.omega1, (t * (LMAX + 1) + l) * C + n);
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) V[l * l + m] = w * Y[l * l + m];
    }
  } else {
    constexpr LayerPlan LP = PlanCT<LMAX, NL>::plan.layer[K - 1];
    float Vin[LP.n_in_comps];
    recompute_V<LMAX, NL, K - 1, C, B16, NG>(a, t, n, Y, Gp, Vin);
#pragma unroll
    for (int q = 0; q < LP.n_out_comps; ++q) V[q] = 0.0f;
    static_for<0, LP.n_paths>([&](auto P) {
      constexpr int k = decltype(P)::value;
      constexpr PathT pt = LP.p[k];
      if constexpr (pt.out_off >= 0) {
        float T[2 * pt.l3 + 1];
        path_fwd<LMAX, NL, K, k>(Vin, Gp[K - 1], T);
        const float al = a.alpha_l[K - 1][k * C + n];
#pragma unroll
        for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) V[pt.out_off + m3] += al * T[m3];
      }
    });
  }
}

// T^pi[m3] = sum over the nonzeros of C^{l1 l2 l3}: C V[m1] Gamma[m2]
template <int LMAX, int NL, int L, int K>
__device__ __forceinline__ void path_fwd(const float* V, const float* G, float* T) {
  constexpr PathT pt = LayerCT<LMAX, NL, L>::lp.p[K];
  constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
#pragma unroll
  for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) T[m3] = 0.0f;
  static_for<0, nz.n>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    T[nz.m3[q]] += nz.c[q] * V[pt.in_off + nz.m1[q]] * G[pt.l2 * pt.l2 + nz.m2[q]];
  });
}

// dE/dV^K (K < NL) of edge t, channel n: the adjoint of layer K + 1's
// products, dE/dV^K[m1] = sum over paths and nonzeros of
// C dE/dT^{K+1}[m3] Gamma^{K+1}[m2], where dE/dT^{K+1} = dE/ds^{K+1} on the
// 0e paths plus alpha^{K+1} dE/dV^{K+1} (rebuilt the same way) on the
// others.  Gn[j] holds Gamma^{L+1+j} (registers).
template <int LMAX, int NL, int L, int K, int C, int NG>
__device__ __forceinline__ void recompute_gV(const TPArgs& a, int64_t t, int n,
                                             const float (&Gn)[NG][(LMAX + 1) * (LMAX + 1)], float* GV) {
  constexpr LayerPlan LP = PlanCT<LMAX, NL>::plan.layer[K];  // layer K + 1
  float GVO[LP.n_out_comps > 0 ? LP.n_out_comps : 1];
  if constexpr (K + 1 < NL) recompute_gV<LMAX, NL, L, K + 1, C, NG>(a, t, n, Gn, GVO);
#pragma unroll
  for (int q = 0; q < LP.n_in_comps; ++q) GV[q] = 0.0f;
  const float* G = Gn[K - L];
  static_for<0, LP.n_paths>([&](auto P) {
    constexpr int k = decltype(P)::value;
    constexpr PathT pt = LP.p[k];
    constexpr int d3 = 2 * pt.l3 + 1;
    constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
    float GT[d3];
#pragma unroll
    for (int m3 = 0; m3 < d3; ++m3) GT[m3] = 0.0f;
    if constexpr (pt.s_idx >= 0) GT[0] = a.gs_l[K][(t * LP.n0e + pt.s_idx) * C + n];
    if constexpr (pt.out_off >= 0) {
      const float al = a.alpha_l[K][k * C + n];
#pragma unroll
      for (int m3 = 0; m3 < d3; ++m3) GT[m3] += al * GVO[pt.out_off + m3];
    }
    static_for<0, nz.n>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      GV[pt.in_off + nz.m1[q]] += nz.c[q] * GT[nz.m3[q]] * G[pt.l2 * pt.l2 + nz.m2[q]];
    });
  });
}

// Layers up to 2 fit 5 wavefronts per SIMD; the deeper rebuild of V^{L-1}
// needs 4 and an edge loop that is not unrolled.
template <int LMAX, int NL, int L, int C, bool B16>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(L >= 3 ? 4 : 5))) k_tp_fwd(TPArgs a) {
  constexpr int UNR = L >= 3 ? 1 : 2;
  constexpr LayerPlan LP = LayerCT<LMAX, NL, L>::lp;
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  constexpr int NS = 256 / C;
  constexpr int NCI = LP.n_in_comps, NCO = LP.n_out_comps > 0 ? LP.n_out_comps : 1;
  __shared__ float red[NS * NLM * C];
  __shared__ float gam[NLM * C];
  const int n = threadIdx.x % C, slot = threadIdx.x / C;
  const int64_t a0 = a.rr.chunk_rows[a.rr.chunk], a1 = a.rr.chunk_rows[a.rr.chunk + 1];
  const int64_t e0 = a.rr.row_ptr[a0];
  for (int64_t i = a0 + blockIdx.x; i < a1; i += gridDim.x) {
    const int64_t eb = a.rr.row_ptr[i], ee = a.rr.row_ptr[i + 1];
    float acc[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) acc[q] = 0.0f;
#pragma unroll UNR
    for (int64_t e = eb + slot; e < ee; e += NS) {
      const int64_t t = e - e0;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        const float w = ld_w<B16>(a.omega, (t * (LMAX + 1) + l) * C + n);
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) acc[l * l + m] += w * Y[l * l + m];
      }
    }
#pragma unroll
    for (int q = 0; q < NLM; ++q) red[(slot * NLM + q) * C + n] = acc[q];
    __syncthreads();
    for (int q = slot; q < NLM; q += NS) {
      float g = 0.0f;
#pragma unroll
      for (int s = 0; s < NS; ++s) g += red[(s * NLM + q) * C + n];
      g *= a.inv_sqrt_nbar;
      gam[q * C + n] = g;
      a.gamma[(i * NLM + q) * C + n] = g;
    }
    __syncthreads();
    float G[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) G[q] = gam[q * C + n];
    float Gp[L > 1 ? L - 1 : 1][NLM];
    load_gammas<LMAX, 0, L - 1, C>(a, i, n, Gp);
#pragma unroll UNR
    for (int64_t e = eb + slot; e < ee; e += NS) {
      const int64_t t = e - e0;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
      float V[NCI];
      recompute_V<LMAX, NL, L - 1, C, B16>(a, t, n, Y, Gp, V);
      // only the scalar (0e) paths leave the kernel; V^L is recomputed by
      // the layers that read it
      static_for<0, LP.n_paths>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr PathT pt = LP.p[k];
        if constexpr (pt.s_idx >= 0) {
          float T[2 * pt.l3 + 1];
          path_fwd<LMAX, NL, L, k>(V, G, T);
          const int64_t si = (t * LP.n0e + pt.s_idx) * C + n;
          st_w<B16>(a.s, si, T[0]);
        }
      });
    }
    __syncthreads();
  }
}

template <int LMAX, int NL, int L, int C, bool B16>
__global__ void __launch_bounds__(256) k_tp_bwd(TPArgs a) {
  constexpr LayerPlan LP = LayerCT<LMAX, NL, L>::lp;
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  constexpr int NS = 256 / C;
  constexpr int NCI = LP.n_in_comps;
  __shared__ float red[NS * NLM * C];
  const int n = threadIdx.x % C, slot = threadIdx.x / C;
  const int64_t a0 = a.rr.chunk_rows[a.rr.chunk], a1 = a.rr.chunk_rows[a.rr.chunk + 1];
  const int64_t e0 = a.rr.row_ptr[a0];
  for (int64_t i = a0 + blockIdx.x; i < a1; i += gridDim.x) {
    const int64_t eb = a.rr.row_ptr[i], ee = a.rr.row_ptr[i + 1];
    float G[NLM], GG[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      G[q] = a.gamma[(i * NLM + q) * C + n];
      GG[q] = 0.0f;
    }
    float Gp[L > 1 ? L - 1 : 1][NLM], Gn[L < NL ? NL - L : 1][NLM];
    load_gammas<LMAX, 0, L - 1, C>(a, i, n, Gp);
    load_gammas<LMAX, L, NL - L, C>(a, i, n, Gn);
    for (int64_t e = eb + slot; e < ee; e += NS) {
      const int64_t t = e - e0;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
      float V[NCI], GV[NCI];
      recompute_V<LMAX, NL, L - 1, C, B16>(a, t, n, Y, Gp, V);
      // dE/dV^L of this edge and channel
      float GVO[LP.n_out_comps > 0 ? LP.n_out_comps : 1];
      if constexpr (L < NL) recompute_gV<LMAX, NL, L, L, C, NL - L>(a, t, n, Gn, GVO);
#pragma unroll
      for (int q = 0; q < NCI; ++q) GV[q] = 0.0f;
      static_for<0, LP.n_paths>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr PathT pt = LP.p[k];
        constexpr int d3 = 2 * pt.l3 + 1;
        constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
        float GT[d3];
#pragma unroll
        for (int m3 = 0; m3 < d3; ++m3) GT[m3] = 0.0f;
        if constexpr (pt.s_idx >= 0) GT[0] = a.gs[(t * LP.n0e + pt.s_idx) * C + n];
        if constexpr (pt.out_off >= 0) {
          const float al = a.alpha[k * C + n];
#pragma unroll
          for (int m3 = 0; m3 < d3; ++m3) GT[m3] += al * GVO[pt.out_off + m3];
        }
        static_for<0, nz.n>([&](auto Q) {
          constexpr int q = decltype(Q)::value;
          const float cg = nz.c[q] * GT[nz.m3[q]];
          GV[pt.in_off + nz.m1[q]] += cg * G[pt.l2 * pt.l2 + nz.m2[q]];
          GG[pt.l2 * pt.l2 + nz.m2[q]] += cg * V[pt.in_off + nz.m1[q]];
        });
      });
      if constexpr (L == 1) {
        // V^0 = omega^1 (x) Y
        float gyc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) gyc[q] = 0.0f;
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
          const float w = ld_w<B16>(a.omega1, (t * (LMAX + 1) + l) * C + n);
          float go = 0.0f;
#pragma unroll
          for (int m = 0; m < 2 * l + 1; ++m) {
            go += GV[l * l + m] * Y[l * l + m];
            gyc[l * l + m] = GV[l * l + m] * w;
          }
          st_w<B16>(a.gomega, (t * (LMAX + 1) + l) * C + n, go);
        }
        add_channel_sums<C, NLM>(gyc, a.gy + t * GEO_STRIDE, n);
      }
    }
    // dE/dGamma summed over the slots, scaled by nbar^-1/2
#pragma unroll
    for (int q = 0; q < NLM; ++q) red[(slot * NLM + q) * C + n] = GG[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      float g = 0.0f;
#pragma unroll
      for (int s = 0; s < NS; ++s) g += red[(s * NLM + q) * C + n];
      GG[q] = g * a.inv_sqrt_nbar;
    }
    for (int64_t e = eb + slot; e < ee; e += NS) {
      const int64_t t = e - e0;
      const float* Y = a.geo + t * GEO_STRIDE + GEO_Y;
      float gyc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) gyc[q] = 0.0f;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        const float w = ld_w<B16>(a.omega, (t * (LMAX + 1) + l) * C + n);
        float go = 0.0f;
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) {
          const float gg = GG[l * l + m];
          go += gg * Y[l * l + m];
          gyc[l * l + m] = gg * w;
        }
        const int64_t gi = (t * (LMAX + 1) + l) * C + n;
        if constexpr (L == 1) go += ld_w<B16>(a.gomega, gi);
        st_w<B16>(a.gomega, gi, go);
      }
      add_channel_sums<C, NLM>(gyc, a.gy + t * GEO_STRIDE, n);
    }
    __syncthreads();
  }
}

typedef void (*tp_kernel_t)(TPArgs);

template <int LMAX, int NL, int C, bool B16>
static tp_kernel_t pick(int L, bool bwd) {
  if (L == 1) return bwd ? k_tp_bwd<LMAX, NL, 1, C, B16> : k_tp_fwd<LMAX, NL, 1, C, B16>;
  if constexpr (NL >= 2) if (L == 2) return bwd ? k_tp_bwd<LMAX, NL, 2, C, B16> : k_tp_fwd<LMAX, NL, 2, C, B16>;
  if constexpr (NL >= 3) if (L == 3) return bwd ? k_tp_bwd<LMAX, NL, 3, C, B16> : k_tp_fwd<LMAX, NL, 3, C, B16>;
  return nullptr;
}

template <int LMAX, int C, bool B16>
static tp_kernel_t pick_nl(int NL, int L, bool bwd) {
  switch (NL) {
    case 1: return pick<LMAX, 1, C, B16>(L, bwd);
    case 2: return pick<LMAX, 2, C, B16>(L, bwd);
    case 3: return pick<LMAX, 3, C, B16>(L, bwd);
  }
  return nullptr;
}

template <int LMAX, bool B16>
static tp_kernel_t pick_c(int C, int NL, int L, bool bwd) {
  switch (C) {
    case 8: return pick_nl<LMAX, 8, B16>(NL, L, bwd);
    case 16: return pick_nl<LMAX, 16, B16>(NL, L, bwd);
    case 32: return pick_nl<LMAX, 32, B16>(NL, L, bwd);
    case 64: return pick_nl<LMAX, 64, B16>(NL, L, bwd);
  }
  return nullptr;
}

template <bool B16>
static tp_kernel_t pick_l(int lmax, int C, int NL, int L, bool bwd) {
  switch (lmax) {
    case 0: return pick_c<0, B16>(C, NL, L, bwd);
    case 1: return pick_c<1, B16>(C, NL, L, bwd);
    case 2: return pick_c<2, B16>(C, NL, L, bwd);
  }
  return nullptr;
}

int launch_tp(int lmax, int NL, int L, int C, bool bwd, bool bf16, const TPArgs& a, int64_t n_atoms_max,
              hipStream_t st) {
  tp_kernel_t k = bf16 ? pick_l<true>(lmax, C, NL, L, bwd) : pick_l<false>(lmax, C, NL, L, bwd);
  if (!k) { set_error("tensor-product kernel not built for this shape"); return AFM_E_UNSUPPORTED; }
  const unsigned grid = grid_for(n_atoms_max, 1, 65536);
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, st, a);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

}  // namespace afm
