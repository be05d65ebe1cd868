// Environment sums and channelwise Clebsch-Gordan tensor products (the
// "tensor features ... l = 2 in full O(3)" of Methodology / Model Training).
//
// One group of C lanes (one lane per channel) per central atom:
//   forward:  Gamma_i[lm][n] = nbar^-1/2 sum_{e in row i} omega_e[l][n] Y_e[lm]
//             T^pi_e[m3][n] = sum C^{l1 l2 l3}[m1][m2][m3] V_e[l1 p1, m1][n] Gamma_i[l2 m2][n]
//             s_e (0e paths), V'_e = sum_pi alpha[pi][n] T^pi_e   (next layer)
//   backward: the adjoints of both lines.
// With the Gammas fixed, an edge's tensor track is linear in its layer-1
// input V^0 = omega^1 (x) Y, so the kernels form small per-atom, per-channel
// linear maps once per row and apply them per edge; per-edge tensor features
// and their adjoints never go to memory.  The products run over the nonzero
// CG entries only, unrolled with immediate coefficients from the
// compile-time tables (cg_ct.h).
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
template <int LMAX, int NL, int K>
struct LayerCT {
  static constexpr LayerPlan lp = PlanCT<LMAX, NL>::plan.layer[K - 1];
};

// A group of C = 64 lanes is one whole wavefront: its atom, edge indices
// and spherical harmonics are then wavefront-uniform and live in SGPRs
// (loaded once by nine lanes and broadcast), which keeps the per-edge
// vector-memory instructions to the per-channel streams.
template <int C>
__device__ __forceinline__ int group_index() {
  if constexpr (C == 64) return __builtin_amdgcn_readfirstlane((int)threadIdx.x) >> 6;
  else return threadIdx.x / C;
}
template <int C>
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  if constexpr (C == 64) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
  } else {
    return v;
  }
}
// Y^{l <= LMAX} of an edge, fetched ahead of its use (the edge loops issue
// the next edge's loads before working on the current one)
// (Y^0..Y^2 in the geometry record, Y^3 in its own for l_max = 3)
template <int C, int NLM>
struct YFetch {
  float v[C == 64 ? 1 : NLM];
  __device__ __forceinline__ void fetch(const TPArgs& a, int64_t t) {
    const float* p = a.geo + t * GEO_STRIDE + GEO_Y;
    if constexpr (C == 64) {
      const int lane = threadIdx.x & 63;
      if constexpr (NLM > 9)
        v[0] = lane < 9 ? p[lane] : (lane < NLM ? a.geo3[t * GEO3_STRIDE + lane - 9] : 0.0f);
      else
        v[0] = lane < NLM ? p[lane] : 0.0f;
    } else {
#pragma unroll
      for (int q = 0; q < NLM; ++q) v[q] = q < 9 ? p[q] : a.geo3[t * GEO3_STRIDE + q - 9];
    }
  }
  __device__ __forceinline__ void get(float (&Y)[NLM]) const {
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      if constexpr (C == 64)
        Y[q] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[0]), q));
      else
        Y[q] = v[q];
    }
  }
};

// accumulator of dE/dY_q of edge t (q >= 9: the l = 3 record)
__device__ __forceinline__ float* gy_slot(const TPArgs& a, int64_t t, int q) {
  return q < 9 ? a.gy + t * GEO_STRIDE + q : a.gy3 + t * GEO3_STRIDE + (q - 9);
}
// the dE/dY accumulators an edge's channel sums are added to (C = 64: lane
// 4k holds value k), fetched ahead like the other per-edge inputs
template <int C, int NV>
struct GyFetch {
  float v;
  __device__ __forceinline__ void fetch(const TPArgs& a, int64_t t, int n) {
    if constexpr (C == 64) v = ((n & 3) == 0 && (n >> 2) < NV) ? *gy_slot(a, t, n >> 2) : 0.0f;
    else v = 0.0f;
  }
};
// dE/dY_q(t) = (fetched) dE/dY_q(t) + sum over the C channels of v[q], q < NV
template <int C, int NV>
__device__ __forceinline__ void add_channel_sums_to(float (&v)[16], const TPArgs& a, int64_t t, int n,
                                                    const GyFetch<C, NV>& old) {
  if constexpr (C == 64) {
    const float y = wave_sum16(v, n);
    if ((n & 3) == 0 && (n >> 2) < NV) *gy_slot(a, t, n >> 2) = old.v + y;
  } else {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const float y = group_sum<C>(v[q]);
      if (n == 0) *gy_slot(a, t, q) += y;
    }
  }
}

// components of V^J (J = 0: the layer-1 inputs omega^1 (x) Y, index l*l+m)
template <int LMAX, int NL, int J>
constexpr int n_comps() {
  if constexpr (J == 0) return (LMAX + 1) * (LMAX + 1);
  else return LayerCT<LMAX, NL, J>::lp.n_out_comps;
}

constexpr int scalar_path_of(const LayerPlan& lp, int s) {
  for (int k = 0; k < lp.n_paths; ++k)
    if (lp.p[k].s_idx == s) return k;
  return -1;
}

// dE/ds inputs of the layer-L adjoint: the scalar slots of layers L..NL,
// layer by layer; slot b belongs to layer slot_layer(b), index slot_sub(b)
template <int LMAX, int NL, int L>
struct Slots {
  static constexpr int count() {
    int n = 0;
    for (int K = L; K <= NL; ++K) n += PlanCT<LMAX, NL>::plan.layer[K - 1].n0e;
    return n;
  }
  static constexpr int layer(int b) {
    for (int K = L; K <= NL; ++K) {
      const int n0 = PlanCT<LMAX, NL>::plan.layer[K - 1].n0e;
      if (b < n0) return K;
      b -= n0;
    }
    return -1;
  }
  static constexpr int sub(int b) {
    for (int K = L; K <= NL; ++K) {
      const int n0 = PlanCT<LMAX, NL>::plan.layer[K - 1].n0e;
      if (b < n0) return b;
      b -= n0;
    }
    return -1;
  }
};

// the scalar path feeding slot S of layer K and the block of V^{K-1} it reads
template <int LMAX, int NL, int K, int S>
struct UnitCT {
  static constexpr PathT pt = LayerCT<LMAX, NL, K>::lp.p[scalar_path_of(LayerCT<LMAX, NL, K>::lp, S)];
  static constexpr int off = pt.in_off, len = 2 * pt.l1 + 1;
};

// Gamma of layers 1..NG of atom i, channel nc (G[K-1] = Gamma^K)
template <int LMAX, int NL, int NG, int CS>
__device__ __forceinline__ void load_gammas(const TPArgs& a, int64_t i, int nc,
                                            float (&G)[NL][(LMAX + 1) * (LMAX + 1)]) {
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
#pragma unroll
  for (int l = 0; l < NG; ++l)
#pragma unroll
    for (int q = 0; q < NLM; ++q) G[l][q] = a.gamma_l[l][(i * NLM + q) * CS + nc];
}

// Layer K forward on given input features: V^K = sum over paths with an
// output of alpha^K (C V^{K-1} Gamma^K).
template <int LMAX, int NL, int K, int CS>
__device__ __forceinline__ void fwd_layer(const TPArgs& a, int nc, const float* G, const float* vin, float* vout) {
  constexpr LayerPlan LP = LayerCT<LMAX, NL, K>::lp;
#pragma unroll
  for (int q = 0; q < LP.n_out_comps; ++q) vout[q] = 0.0f;
  static_for<0, LP.n_paths>([&](auto P) {
    constexpr int k = decltype(P)::value;
    constexpr PathT pt = LP.p[k];
    if constexpr (pt.out_off >= 0) {
      constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
      float T[2 * pt.l3 + 1];
#pragma unroll
      for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) T[m3] = 0.0f;
      static_for<0, nz.n>([&](auto Q) {
        constexpr int q = decltype(Q)::value;
        T[nz.m3[q]] += nz.c[q] * vin[pt.in_off + nz.m1[q]] * G[pt.l2 * pt.l2 + nz.m2[q]];
      });
      const float al = a.alpha_l[K - 1][k * CS + nc];
#pragma unroll
      for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) vout[pt.out_off + m3] += al * T[m3];
    }
  });
}

// V^J for given V^0 (layers 1..J forward)
template <int LMAX, int NL, int J, int CS>
__device__ __forceinline__ void fwd_chain(const TPArgs& a, int nc, const float (&G)[NL][(LMAX + 1) * (LMAX + 1)],
                                          const float* v0, float* vJ) {
  if constexpr (J == 0) {
#pragma unroll
    for (int q = 0; q < (LMAX + 1) * (LMAX + 1); ++q) vJ[q] = v0[q];
  } else {
    float vin[n_comps<LMAX, NL, J - 1>()];
    fwd_chain<LMAX, NL, J - 1, CS>(a, nc, G, v0, vin);
    fwd_layer<LMAX, NL, J, CS>(a, nc, G[J - 1], vin, vJ);
  }
}

// Adjoint of layer K's mixing and products: dE/dV^{K-1} from dE/dV^K,
// where dE/dV^K is nonzero only on components [OFF, OFF + LEN).
template <int LMAX, int NL, int K, int OFF, int LEN, int CS>
__device__ __forceinline__ void adj_layer(const TPArgs& a, int nc, const float* G, const float* gvo, float* gv) {
  constexpr LayerPlan LP = LayerCT<LMAX, NL, K>::lp;
#pragma unroll
  for (int q = 0; q < LP.n_in_comps; ++q) gv[q] = 0.0f;
  static_for<0, LP.n_paths>([&](auto P) {
    constexpr int k = decltype(P)::value;
    constexpr PathT pt = LP.p[k];
    if constexpr (pt.out_off >= OFF && pt.out_off < OFF + LEN) {
      constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
      const float al = a.alpha_l[K - 1][k * CS + nc];
      float GT[2 * pt.l3 + 1];
#pragma unroll
      for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) GT[m3] = al * gvo[pt.out_off + m3];
      static_for<0, nz.n>([&](auto Q) {
        constexpr int q = decltype(Q)::value;
        gv[pt.in_off + nz.m1[q]] += nz.c[q] * GT[nz.m3[q]] * G[pt.l2 * pt.l2 + nz.m2[q]];
      });
    }
  });
}

// dE/dV^J (dense) from dE/dV^M (nonzero on [OFF, OFF + LEN)), J < M
template <int LMAX, int NL, int M, int J, int OFF, int LEN, int CS>
__device__ __forceinline__ void adj_down(const TPArgs& a, int nc, const float (&G)[NL][(LMAX + 1) * (LMAX + 1)],
                                         const float* gM, float* gJ) {
  if constexpr (M - 1 == J) {
    adj_layer<LMAX, NL, M, OFF, LEN, CS>(a, nc, G[M - 1], gM, gJ);
  } else {
    float t[n_comps<LMAX, NL, M - 1>()];
    adj_layer<LMAX, NL, M, OFF, LEN, CS>(a, nc, G[M - 1], gM, t);
    adj_down<LMAX, NL, M - 1, J, 0, n_comps<LMAX, NL, M - 1>(), CS>(a, nc, G, t, gJ);
  }
}

// dE/dV^{K-1} for dE/ds = 1 on scalar slot S of layer K: C Gamma^K on the
// block [UnitCT::off, + len) of the path's input irrep (other entries unset)
template <int LMAX, int NL, int K, int S>
__device__ __forceinline__ void unit_inject(const float* G, float* g) {
  using U = UnitCT<LMAX, NL, K, S>;
  constexpr PathT pt = U::pt;
  constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, 0>::nz;
#pragma unroll
  for (int m = 0; m < U::len; ++m) g[U::off + m] = 0.0f;
  static_for<0, nz.n>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    g[pt.in_off + nz.m1[q]] += nz.c[q] * G[pt.l2 * pt.l2 + nz.m2[q]];
  });
}

// dE/dGamma^L += sum over layer L's paths of C (dE/dT^L) X, with
// dE/dT^L = alpha^L dE/dV^L (dV nonzero on [OFF, OFF + LEN)) and X given
// input features; with WANT_D also the products' adjoint in their input,
// D += C (dE/dT^L) Gamma^L.
template <int LMAX, int NL, int L, int OFF, int LEN, bool WANT_D, int CS>
__device__ __forceinline__ void contract(const TPArgs& a, int nc, const float* G, const float* dv, const float* X,
                                         float* GG, float* D) {
  constexpr LayerPlan LP = LayerCT<LMAX, NL, L>::lp;
  static_for<0, LP.n_paths>([&](auto P) {
    constexpr int k = decltype(P)::value;
    constexpr PathT pt = LP.p[k];
    if constexpr (pt.out_off >= OFF && pt.out_off < OFF + LEN) {
      constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, pt.l3>::nz;
      const float al = a.alpha_l[L - 1][k * CS + nc];
      float GT[2 * pt.l3 + 1];
#pragma unroll
      for (int m3 = 0; m3 < 2 * pt.l3 + 1; ++m3) GT[m3] = al * dv[pt.out_off + m3];
      static_for<0, nz.n>([&](auto Q) {
        constexpr int q = decltype(Q)::value;
        const float cg = nz.c[q] * GT[nz.m3[q]];
        GG[pt.l2 * pt.l2 + nz.m2[q]] += cg * X[pt.in_off + nz.m1[q]];
        if constexpr (WANT_D) D[pt.in_off + nz.m1[q]] += cg * G[pt.l2 * pt.l2 + nz.m2[q]];
      });
    }
  });
}

// Given the Gammas, the tensor track of an edge is linear in its layer-1
// input V^0 = omega^1 (x) Y: V^L = R^L V^0 and s^L = P^L V^0 with per-atom,
// per-channel matrices (products with fixed Gammas, then channelwise
// mixing).  The kernels therefore form these small maps once per atom and
// apply them per edge, instead of running every earlier (forward) or later
// (adjoint) layer's products again for each edge.
//
// One group of C lanes per central atom (lane = channel), 256 / C atoms per
// workgroup; a group walks all edges of its row, so the row sums need no
// cross-lane reduction and no LDS.
// occupancy floor of the forward kernels: their edge loops are chains of
// small dependent loads, so more wavefronts per SIMD hide more latency
// (layer 3 of three at l_max = 2: 115 VGPRs / 4 waves -> 6 waves, 12 %
// faster); l_max = 3 keeps the compiler's choice
template <int LMAX>
constexpr int tp_fwd_waves() { return LMAX <= 2 ? 6 : 1; }

template <int LMAX, int NL, int L, int C, bool B16, int CS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(tp_fwd_waves<LMAX>()))) k_tp_fwd(TPArgs a) {
  constexpr LayerPlan LP = LayerCT<LMAX, NL, L>::lp;
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  constexpr int NA = 256 / C;
  constexpr int NS0 = LP.n0e;
  const int n = threadIdx.x % C, grp = group_index<C>();
  const int nc = a.c0 + n;   // channel in the arrays (a launch covers channels [c0, c0 + C))
  const int64_t a0 = a.rr.chunk_rows[a.rr.chunk], a1 = a.rr.chunk_rows[a.rr.chunk + 1];
  const int64_t e0 = uniform64<C>(a.rr.row_ptr[a0]);
  // per-edge inputs: Y and one omega (omega^L for Gamma^L, omega^1 for V^0)
  struct EdgeIn {
    YFetch<C, NLM> y;
    float w[LMAX + 1];
  };
  auto fetch = [&](int64_t t, const void* om, EdgeIn& x) {
    x.y.fetch(a, t);
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) x.w[l] = ld_w<B16>(om, (t * (LMAX + 1) + l) * CS + nc);
  };
  for (int64_t i = a0 + (int64_t)blockIdx.x * NA + grp; i < a1; i += (int64_t)gridDim.x * NA) {
    const int64_t eb = uniform64<C>(a.rr.row_ptr[i]), ee = uniform64<C>(a.rr.row_ptr[i + 1]);
    float G[NL][NLM];
    // Gamma^L_i = nbar^-1/2 sum over the row of omega^L (x) Y
#pragma unroll
    for (int q = 0; q < NLM; ++q) G[L - 1][q] = 0.0f;
    {
      EdgeIn cur, nxt;
      if (eb < ee) fetch(eb - e0, a.omega, cur);
      nxt = cur;
      for (int64_t e = eb; e < ee; ++e) {
        const int64_t t = e - e0;
        if (e + 1 < ee) fetch(t + 1, a.omega, nxt);
        float Y[NLM];
        cur.y.get(Y);
#pragma unroll
        for (int l = 0; l <= LMAX; ++l)
#pragma unroll
          for (int m = 0; m < 2 * l + 1; ++m) G[L - 1][l * l + m] += cur.w[l] * Y[l * l + m];
        cur = nxt;
      }
    }
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      G[L - 1][q] *= a.inv_sqrt_nbar;
      a.gamma[(i * NLM + q) * CS + nc] = G[L - 1][q];
    }
    load_gammas<LMAX, NL, L - 1, CS>(a, i, nc, G);
    // rows of P^L: dE/dV^0 for a unit dE/ds on each scalar path (layer L's
    // products, then the earlier layers' adjoints); for L = 1 a row is the
    // path's C Gamma^1 block
    float P[NS0 > 0 ? NS0 : 1][NLM];
    static_for<0, NS0>([&](auto SS) {
      constexpr int S = decltype(SS)::value;
      if constexpr (L == 1) {
        unit_inject<LMAX, NL, 1, S>(G[0], P[S]);
      } else {
        using U = UnitCT<LMAX, NL, L, S>;
        float gb[n_comps<LMAX, NL, L - 1>()];
        unit_inject<LMAX, NL, L, S>(G[L - 1], gb);
        adj_down<LMAX, NL, L - 1, 0, U::off, U::len, CS>(a, nc, G, gb, P[S]);
      }
    });
    EdgeIn cur, nxt;
    if (eb < ee) fetch(eb - e0, a.omega1, cur);
    nxt = cur;
    for (int64_t e = eb; e < ee; ++e) {
      const int64_t t = e - e0;
      if (e + 1 < ee) fetch(t + 1, a.omega1, nxt);
      float Y[NLM];
      cur.y.get(Y);
      float V0[NLM];
#pragma unroll
      for (int l = 0; l <= LMAX; ++l)
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) V0[l * l + m] = cur.w[l] * Y[l * l + m];
      static_for<0, NS0>([&](auto SS) {
        constexpr int S = decltype(SS)::value;
        using U = UnitCT<LMAX, NL, L, S>;
        constexpr int q0 = L == 1 ? U::off : 0, q1 = L == 1 ? U::off + U::len : NLM;
        float s = 0.0f;
#pragma unroll
        for (int q = q0; q < q1; ++q) s += P[S][q] * V0[q];
        st_w<B16>(a.s, (t * NS0 + S) * CS + nc, s);
      });
      cur = nxt;
    }
  }
}

// Adjoint of layer L.  With g'_e the edge's dE/ds of layers L..NL (the
// slots), dE/dT^L_e and V^{L-1}_e are linear in g'_e and V^0_e, so
// dE/dGamma^L needs only the row moment M = sum_e V^0_e g'_e^T: each slot b
// contributes the layer-L product adjoint of (its unit dE/dT^L) with
// R^{L-1} M[:, b].  Layer 1 also needs dE/dV^0_e = D g'_e per edge (D: the
// rows of every layer's P, formed alongside).
// occupancy floor of the adjoint kernels (register budget 512 / waves),
// per layer by A/B on the three-layer step (the last layer's lighter
// adjoint gains from a fifth wavefront, the middle one loses)
template <int LMAX, int NL, int L>
constexpr int tp_bwd_waves() { return LMAX == 3 ? 2 : (L == NL && NL >= 3) ? 5 : 4; }

template <int LMAX, int NL, int L, int C, bool B16, int CS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(tp_bwd_waves<LMAX, NL, L>())))
k_tp_bwd(TPArgs a) {
  constexpr int NLM = (LMAX + 1) * (LMAX + 1);
  constexpr int NA = 256 / C;
  using SL = Slots<LMAX, NL, L>;
  constexpr int NB = SL::count();
  const int n = threadIdx.x % C, grp = group_index<C>();
  const int nc = a.c0 + n;   // channel in the arrays (a launch covers channels [c0, c0 + C))
  const int64_t a0 = a.rr.chunk_rows[a.rr.chunk], a1 = a.rr.chunk_rows[a.rr.chunk + 1];
  const int64_t e0 = uniform64<C>(a.rr.row_ptr[a0]);
  // dE/ds of slot b for edge t
  auto load_slots = [&](int64_t t, float (&gp)[NB]) {
    static_for<0, NB>([&](auto B) {
      constexpr int b = decltype(B)::value;
      constexpr int K = SL::layer(b), S = SL::sub(b);
      constexpr int n0 = LayerCT<LMAX, NL, K>::lp.n0e;
      gp[b] = ld_w<B16>(a.gs_l[K - 1], (t * n0 + S) * CS + nc);
    });
  };
  // per-edge inputs of the moment pass and of the dE/domega pass
  struct In1 {
    YFetch<C, NLM> y;
    float w[LMAX + 1], gp[NB];
  };
  struct In3 {
    YFetch<C, NLM> y;
    float w[LMAX + 1], gp[L == 1 ? NB : 1];
    GyFetch<C, NLM> gy;
  };
  auto fetch1 = [&](int64_t t, In1& x) {
    x.y.fetch(a, t);
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) x.w[l] = ld_w<B16>(a.omega1, (t * (LMAX + 1) + l) * CS + nc);
    load_slots(t, x.gp);
  };
  auto fetch3 = [&](int64_t t, In3& x) {
    x.y.fetch(a, t);
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) x.w[l] = ld_w<B16>(a.omega, (t * (LMAX + 1) + l) * CS + nc);
    if constexpr (L == 1) load_slots(t, x.gp);
    x.gy.fetch(a, t, n);
  };
  for (int64_t i = a0 + (int64_t)blockIdx.x * NA + grp; i < a1; i += (int64_t)gridDim.x * NA) {
    const int64_t eb = uniform64<C>(a.rr.row_ptr[i]), ee = uniform64<C>(a.rr.row_ptr[i + 1]);
    // row moment M[a][b] = sum_e V^0_e[a] g'_e[b]
    float M[NLM][NB];
#pragma unroll
    for (int q = 0; q < NLM; ++q)
#pragma unroll
      for (int b = 0; b < NB; ++b) M[q][b] = 0.0f;
    {
      In1 cur, nxt;
      if (eb < ee) fetch1(eb - e0, cur);
      nxt = cur;
      for (int64_t e = eb; e < ee; ++e) {
        const int64_t t = e - e0;
        if (e + 1 < ee) fetch1(t + 1, nxt);
        float Y[NLM];
        cur.y.get(Y);
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
#pragma unroll
          for (int m = 0; m < 2 * l + 1; ++m) {
            const float v = cur.w[l] * Y[l * l + m];
#pragma unroll
            for (int b = 0; b < NB; ++b) M[l * l + m][b] += v * cur.gp[b];
          }
        }
        cur = nxt;
      }
    }
    float G[NL][NLM];
    load_gammas<LMAX, NL, NL, CS>(a, i, nc, G);
    float GG[NLM], D[NLM][NB];
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
      GG[q] = 0.0f;
#pragma unroll
      for (int b = 0; b < NB; ++b) D[q][b] = 0.0f;
    }
    static_for<0, NB>([&](auto B) {
      constexpr int b = decltype(B)::value;
      constexpr int K = SL::layer(b), S = SL::sub(b);
      using U = UnitCT<LMAX, NL, K, S>;
      float m0[NLM];
#pragma unroll
      for (int q = 0; q < NLM; ++q) m0[q] = M[q][b];
      float X[n_comps<LMAX, NL, L - 1>()];
      fwd_chain<LMAX, NL, L - 1, CS>(a, nc, G, m0, X);
      if constexpr (K == L) {
        // unit dE/dT on the scalar path itself: C X on its block
        constexpr PathT pt = U::pt;
        constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, 0>::nz;
        static_for<0, nz.n>([&](auto Q) {
          constexpr int q = decltype(Q)::value;
          GG[pt.l2 * pt.l2 + nz.m2[q]] += nz.c[q] * X[pt.in_off + nz.m1[q]];
        });
      } else {
        float gb[n_comps<LMAX, NL, K - 1>()], Dc[NLM];
#pragma unroll
        for (int q = 0; q < NLM; ++q) Dc[q] = 0.0f;
        unit_inject<LMAX, NL, K, S>(G[K - 1], gb);
        if constexpr (K - 1 == L) {
          contract<LMAX, NL, L, U::off, U::len, L == 1, CS>(a, nc, G[L - 1], gb, X, GG, Dc);
        } else {
          float dv[n_comps<LMAX, NL, L>() > 0 ? n_comps<LMAX, NL, L>() : 1];
          adj_down<LMAX, NL, K - 1, L, U::off, U::len, CS>(a, nc, G, gb, dv);
          contract<LMAX, NL, L, 0, n_comps<LMAX, NL, L>(), L == 1, CS>(a, nc, G[L - 1], dv, X, GG, Dc);
        }
        if constexpr (L == 1) {
#pragma unroll
          for (int q = 0; q < NLM; ++q) D[q][b] = Dc[q];
        }
      }
    });
#pragma unroll
    for (int q = 0; q < NLM; ++q) GG[q] *= a.inv_sqrt_nbar;
    // per edge: dE/domega^L (Gamma^L's adjoint; for L = 1 also V^0's) and
    // the channel sums of dE/dY
    In3 cur, nxt;
    if (eb < ee) fetch3(eb - e0, cur);
    nxt = cur;
    for (int64_t e = eb; e < ee; ++e) {
      const int64_t t = e - e0;
      if (e + 1 < ee) fetch3(t + 1, nxt);
      float Y[NLM];
      cur.y.get(Y);
      float tot[NLM];
#pragma unroll
      for (int q = 0; q < NLM; ++q) tot[q] = GG[q];
      if constexpr (L == 1) {
        const float (&gp)[NB] = cur.gp;
        static_for<0, NB>([&](auto B) {
          constexpr int b = decltype(B)::value;
          constexpr int K = SL::layer(b), S = SL::sub(b);
          if constexpr (K == 1) {
            using U = UnitCT<LMAX, NL, 1, S>;
            constexpr PathT pt = U::pt;
            constexpr ct::Nz nz = ct::NzCT<pt.l1, pt.l2, 0>::nz;
            static_for<0, nz.n>([&](auto Q) {
              constexpr int q = decltype(Q)::value;
              tot[pt.in_off + nz.m1[q]] += nz.c[q] * G[0][pt.l2 * pt.l2 + nz.m2[q]] * gp[b];
            });
          } else {
#pragma unroll
            for (int q = 0; q < NLM; ++q) tot[q] += D[q][b] * gp[b];
          }
        });
      }
      float gyc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) gyc[q] = 0.0f;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        float go = 0.0f;
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) {
          go += tot[l * l + m] * Y[l * l + m];
          gyc[l * l + m] = tot[l * l + m] * cur.w[l];
        }
        st_w<B16>(a.gomega, (t * (LMAX + 1) + l) * CS + nc, go);
      }
      add_channel_sums_to<C, NLM>(gyc, a, t, n, cur.gy);
      cur = nxt;
    }
  }
}

typedef void (*tp_kernel_t)(TPArgs);

template <int LMAX, int NL, int C, bool B16, int CS>
static tp_kernel_t pick(int L, bool bwd) {
  if (L == 1) return bwd ? k_tp_bwd<LMAX, NL, 1, C, B16, CS> : k_tp_fwd<LMAX, NL, 1, C, B16, CS>;
  if constexpr (NL >= 2) if (L == 2) return bwd ? k_tp_bwd<LMAX, NL, 2, C, B16, CS> : k_tp_fwd<LMAX, NL, 2, C, B16, CS>;
  if constexpr (NL >= 3) if (L == 3) return bwd ? k_tp_bwd<LMAX, NL, 3, C, B16, CS> : k_tp_fwd<LMAX, NL, 3, C, B16, CS>;
  return nullptr;
}

// C: channels per launch (threads' channel groups); CS: channels in the arrays
template <int LMAX, int C, bool B16, int CS>
static tp_kernel_t pick_nl(int NL, int L, bool bwd) {
  switch (NL) {
    case 1: return pick<LMAX, 1, C, B16, CS>(L, bwd);
    case 2: return pick<LMAX, 2, C, B16, CS>(L, bwd);
    case 3: return pick<LMAX, 3, C, B16, CS>(L, bwd);
  }
  return nullptr;
}

template <int LMAX, bool B16>
static tp_kernel_t pick_c(int C, int NL, int L, bool bwd) {
  switch (C) {
    case 8: return pick_nl<LMAX, 8, B16, 8>(NL, L, bwd);
    case 16: return pick_nl<LMAX, 16, B16, 16>(NL, L, bwd);
    case 32: return pick_nl<LMAX, 32, B16, 32>(NL, L, bwd);
    case 64: return pick_nl<LMAX, 64, B16, 64>(NL, L, bwd);
    case 128: return pick_nl<LMAX, 64, B16, 128>(NL, L, bwd);
  }
  return nullptr;
}

// l_max = 3: one or two layers, 16 or 64 channels
template <bool B16>
static tp_kernel_t pick_c3(int C, int NL, int L, bool bwd) {
  if (NL == 1) return C == 16 ? pick<3, 1, 16, B16, 16>(L, bwd) : C == 64 ? pick<3, 1, 64, B16, 64>(L, bwd) : nullptr;
  if (NL == 2) return C == 16 ? pick<3, 2, 16, B16, 16>(L, bwd) : C == 64 ? pick<3, 2, 64, B16, 64>(L, bwd) : nullptr;
  return nullptr;
}

template <bool B16>
static tp_kernel_t pick_l(int lmax, int C, int NL, int L, bool bwd) {
  switch (lmax) {
    case 0: return pick_c<0, B16>(C, NL, L, bwd);
    case 1: return pick_c<1, B16>(C, NL, L, bwd);
    case 2: return pick_c<2, B16>(C, NL, L, bwd);
    case 3: return pick_c3<B16>(C, NL, L, bwd);
  }
  return nullptr;
}

// 128 channels run as two consecutive launches of 64-channel kernels over
// the channel groups (the products are channelwise); the per-edge sums over
// channels (dE/dY) accumulate group after group in a fixed order.
int launch_tp(int lmax, int NL, int L, int C, bool bwd, bool bf16, const TPArgs& a, int64_t n_atoms_max,
              hipStream_t st) {
  const int CK = C > 64 ? 64 : C;
  tp_kernel_t k = bf16 ? pick_l<true>(lmax, C, NL, L, bwd) : pick_l<false>(lmax, C, NL, L, bwd);
  if (!k) { set_error("tensor-product kernel not built for this shape"); return AFM_E_UNSUPPORTED; }
  const unsigned grid = grid_for(n_atoms_max, 256 / CK, 65536);
  for (int c0 = 0; c0 < C; c0 += CK) {
    TPArgs ag = a;
    ag.c0 = c0;
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, st, ag);
  }
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

}  // namespace afm
