// BF16 MFMA chains for the per-edge MLPs (gfx950, v_mfma_f32_16x16x32_bf16,
// FP32 accumulation): the two-body MLP, the linear environment embeddings and
// the latent MLPs with their residual updates (Methodology / Model Training:
// two-body latent MLP, "embedding MLP ... linear projection", latent MLP,
// SiLU), forward and adjoint.
//
// Mapping.  Each layer is computed transposed, Y^T = W X^T: the weights are
// the MFMA A operand (16 output features x 32 input features per fragment)
// and a wavefront's edges are the B/C columns (JW blocks of 16 edges).  The
// C result of one layer becomes the B operand of the next without leaving
// registers: lane group g of a 16-row output block holds features 4g..4g+3,
// so a 32-feature input block is fed as k-slots (g, i) <-> feature
//   phi(kb, g, i) = 32 kb + 4 g + (i & 3) + 16 (i >> 2),
// and every weight fragment is packed on the host with the same permutation
// (MFMA pairs A and B k-slots identically, so the product is unchanged).
// Every weight is held as an unevaluated sum of two bf16 numbers (hi + lo,
// lo = bf16(w - hi)) and each fragment product is issued as two MFMAs into
// the same FP32 accumulator, so the weights keep ~16 mantissa bits while
// activations are rounded to bf16 once per layer.  Rounding the weights
// alone would perturb the model itself, an error common to every edge that
// does not average out over a structure; activation rounding is independent
// per edge.  Pre-activations are stored as bf16 in a tile-native layout read
// back by the adjoint.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "device_util.h"
#include "edge_layout.h"
#include "internal.h"

namespace afm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int JW = 2;             // 16-edge column blocks per wavefront
constexpr int TILE = 16 * JW;     // edges per wavefront
constexpr int WAVES = 4;          // wavefronts per workgroup
constexpr int kSplit = 2;         // bf16 terms per weight (hi, lo)

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// host packing

static uint16_t bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// M(r, k) = transpose ? W[k * R + r] : W[r * K + k]; fragments
// [RB][KB][2][64][8] with the hi part of the weight pairs first, lo second
static void pack_matrix(const double* W, int R, int K, bool transpose, std::vector<char>& out,
                        int64_t* off) {
  const int RB = cdiv(R, 16), KB = cdiv(K, 32);
  int64_t o = (int64_t)out.size();
  o = (o + 255) & ~int64_t(255);
  out.resize(o + (int64_t)RB * KB * kSplit * 64 * 16, 0);
  uint16_t* p = reinterpret_cast<uint16_t*>(out.data() + o);
  for (int rb = 0; rb < RB; ++rb)
    for (int kb = 0; kb < KB; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = 16 * rb + (lane & 15), g = lane >> 4;
        for (int i = 0; i < 8; ++i) {
          const int k = 32 * kb + 4 * g + (i & 3) + 16 * (i >> 2);
          double v = 0.0;
          if (r < R && k < K) v = transpose ? W[(int64_t)k * R + r] : W[(int64_t)r * K + k];
          const uint16_t hi = bf16_rne((float)v);
          const uint16_t lo = bf16_rne((float)(v - bf16_value(hi)));
          const int64_t base = (((int64_t)rb * KB + kb) * kSplit * 64 + lane) * 8 + i;
          p[base] = hi;
          p[base + 64 * 8] = lo;
        }
      }
  *off = o;
}

static const afm_param_block* blk(const afm_model* m, const char* name) {
  for (auto& b : m->blocks)
    if (strcmp(b.name, name) == 0) return &b;
  return nullptr;
}

struct FragOffsets {
  int64_t tbf[kMaxTwobody], tbb[kMaxTwobody];
  int64_t envf[kMaxLayers], envb[kMaxLayers];
  int64_t latf[kMaxLayers][kMaxDepth], latb[kMaxLayers][kMaxDepth];
};

// Packs every MFMA weight matrix of the model (forward W and adjoint W^T)
// from the flat float64 weight vector `base`; records byte offsets.
void pack_bf16_frags(const afm_model* m, const double* base, std::vector<char>& out, DevWeights* Wd) {
  const ModelDims& d = m->dims;
  FragOffsets fo{};
  out.clear();
  char nm[32];
  for (int k = 1; k < d.ntb; ++k) {
    snprintf(nm, sizeof nm, "twobody.%d", k);
    const afm_param_block* b = blk(m, nm);
    pack_matrix(base + b->offset, (int)b->rows, (int)b->cols, false, out, &fo.tbf[k]);
    pack_matrix(base + b->offset, (int)b->cols, (int)b->rows, true, out, &fo.tbb[k]);
  }
  for (int L = 1; L <= d.NL; ++L) {
    snprintf(nm, sizeof nm, "layer%d.env", L);
    const afm_param_block* b = blk(m, nm);
    std::vector<double> perm((size_t)b->rows * b->cols);
    for (int l = 0; l <= d.lmax; ++l)
      for (int n = 0; n < d.c; ++n)
        memcpy(&perm[((size_t)l * d.c + n) * d.w], base + b->offset + ((size_t)n * (d.lmax + 1) + l) * d.w,
               sizeof(double) * d.w);
    pack_matrix(perm.data(), (int)b->rows, d.w, false, out, &fo.envf[L - 1]);
    pack_matrix(perm.data(), d.w, (int)b->rows, true, out, &fo.envb[L - 1]);
    for (int k = 0; k < d.depth; ++k) {
      snprintf(nm, sizeof nm, "layer%d.latent.%d", L, k);
      b = blk(m, nm);
      pack_matrix(base + b->offset, (int)b->rows, (int)b->cols, false, out, &fo.latf[L - 1][k]);
      pack_matrix(base + b->offset, (int)b->cols, (int)b->rows, true, out, &fo.latb[L - 1][k]);
    }
  }
  static_assert(sizeof(FragOffsets) <= sizeof(Wd->frag_off), "offset table too small");
  memcpy(Wd->frag_off, &fo, sizeof fo);
}

// ---------------------------------------------------------------------------
// device building blocks

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sigm(float a) { return __builtin_amdgcn_rcpf(1.0f + __expf(-a)); }

__device__ __forceinline__ bf16x8 pack8(f32x4 lo, f32x4 hi) {
  bf16x8 r;
  r[0] = (__bf16)lo[0]; r[1] = (__bf16)lo[1]; r[2] = (__bf16)lo[2]; r[3] = (__bf16)lo[3];
  r[4] = (__bf16)hi[0]; r[5] = (__bf16)hi[1]; r[6] = (__bf16)hi[2]; r[7] = (__bf16)hi[3];
  return r;
}

__device__ __forceinline__ f32x4 ld4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }
__device__ __forceinline__ void st4(float* p, f32x4 v) { *reinterpret_cast<f32x4*>(p) = v; }

// pre-activation tile storage: [tile][RB][JW][64 lanes][4] bf16
__device__ __forceinline__ void st_pre(uint2* pre, int64_t tile, int RB, int rb, int j, int lane, f32x4 v) {
  bf16x4 h;
  h[0] = (__bf16)v[0]; h[1] = (__bf16)v[1]; h[2] = (__bf16)v[2]; h[3] = (__bf16)v[3];
  pre[((tile * RB + rb) * JW + j) * 64 + lane] = __builtin_bit_cast(uint2, h);
}
__device__ __forceinline__ f32x4 ld_pre(const uint2* pre, int64_t tile, int RB, int rb, int j, int lane) {
  bf16x4 h = __builtin_bit_cast(bf16x4, pre[((tile * RB + rb) * JW + j) * 64 + lane]);
  f32x4 v;
  v[0] = (float)h[0]; v[1] = (float)h[1]; v[2] = (float)h[2]; v[3] = (float)h[3];
  return v;
}

// acc (C layout, RB row blocks) -> B fragments of the next layer
template <int RB>
__device__ __forceinline__ void to_frags(const f32x4 (&h)[RB][JW], bf16x8 (&o)[cdiv(RB, 2)][JW]) {
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < cdiv(RB, 2); ++kb)
#pragma unroll
    for (int j = 0; j < JW; ++j) o[kb][j] = pack8(h[2 * kb][j], (2 * kb + 1 < RB) ? h[2 * kb + 1][j] : z);
}

template <int RB>
__device__ __forceinline__ void zero(f32x4 (&a)[RB][JW]) {
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int j = 0; j < JW; ++j) a[rb][j] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Weight fragments are staged through LDS, one k-block (RB hi/lo fragment
// pairs of 2 KB) per stage, double buffered: every wavefront of the workgroup loads a
// share of stage kb+1 into registers while the MFMAs of stage kb run, then
// writes it to the other buffer.  All wavefronts of a workgroup call the
// GEMMs with the same shapes (barriers inside).
constexpr int kStageMax = 16;                 // row blocks per stage (RB <= 16)
constexpr int kFragPerRB = kSplit * 64;       // uint4 per (row block, k-block)
struct Stage {
  uint4 buf[2][kStageMax * kFragPerRB];
};

template <int RB>
constexpr int stage_regs() { return cdiv(RB * kFragPerRB, 256); }

template <int RB, int KB, int R0>
__device__ __forceinline__ void stage_load(const uint4* __restrict__ W, int kb, uint4 (&reg)[stage_regs<RB>()],
                                           int tid) {
#pragma unroll
  for (int q = 0; q < stage_regs<RB>(); ++q) {
    // clamped rather than predicated: the loads stay unconditional, so the
    // staging registers never leave the register file
    const int idx = min(tid + 256 * q, RB * kFragPerRB - 1);
    reg[q] = W[((int64_t)(R0 + idx / kFragPerRB) * KB + kb) * kFragPerRB + (idx % kFragPerRB)];
  }
}
template <int RB>
__device__ __forceinline__ void stage_store(uint4* __restrict__ dst, const uint4 (&reg)[stage_regs<RB>()], int tid) {
#pragma unroll
  for (int q = 0; q < stage_regs<RB>(); ++q) {
    const int idx = tid + 256 * q;
    if (idx < RB * kFragPerRB) dst[idx] = reg[q];
  }
}

// acc[rb] = sum_kb W[R0 + rb][kb] x B(kb) for rb < RB; B(kb, j) supplies
// the B fragments (registers or memory)
template <int RB, int KB, int R0, class BF>
__device__ __forceinline__ void gemm_lds(const uint4* __restrict__ W, Stage& S, BF bfrag, f32x4 (&acc)[RB][JW],
                                         int lane, int tid) {
  static_assert(RB <= kStageMax, "stage too small");
  zero(acc);
  uint4 reg[stage_regs<RB>()];
  stage_load<RB, KB, R0>(W, 0, reg, tid);
  stage_store<RB>(S.buf[0], reg, tid);
  __syncthreads();
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb + 1 < KB) stage_load<RB, KB, R0>(W, kb + 1, reg, tid);
    bf16x8 b[JW];
#pragma unroll
    for (int j = 0; j < JW; ++j) b[j] = bfrag(kb, j);
    const uint4* cur = S.buf[kb & 1];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int h = 0; h < kSplit; ++h) {
        const bf16x8 a = __builtin_bit_cast(bf16x8, cur[rb * kFragPerRB + h * 64 + lane]);
#pragma unroll
        for (int j = 0; j < JW; ++j) acc[rb][j] = mfma(a, b[j], acc[rb][j]);
      }
    }
    if (kb + 1 < KB) stage_store<RB>(S.buf[(kb + 1) & 1], reg, tid);
    __syncthreads();
  }
}

// B fragments held in registers
template <int KB>
struct RegB {
  const bf16x8 (&in)[KB][JW];
  __device__ __forceinline__ bf16x8 operator()(int kb, int j) const { return in[kb][j]; }
};

// B fragment of features [32 kb, 32 kb + 32) of a float32 row-major matrix
// X[t][ld] restricted to columns < kpart (zeros beyond, and for invalid t)
__device__ __forceinline__ bf16x8 ld_frag32(const float* __restrict__ X, int ld, int64_t t, bool valid, int kb,
                                            int kpart, int g) {
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  const int fa = 32 * kb + 4 * g, fb = fa + 16;
  f32x4 lo = (valid && fa + 4 <= kpart) ? ld4(X + t * ld + fa) : z;
  f32x4 hi = (valid && fb + 4 <= kpart) ? ld4(X + t * ld + fb) : z;
  return pack8(lo, hi);
}

// B fragments of [x | s] (x: [t][WX], s: [t][KS], float32) from memory
template <int WX, int KS>
struct CatB {
  const float* x;
  const float* s;
  const int64_t* t;
  const bool* valid;
  int g;
  __device__ __forceinline__ bf16x8 operator()(int kb, int j) const {
    if (32 * kb < WX) return ld_frag32(x, WX, t[j], valid[j], kb, WX, g);
    return ld_frag32(s, KS, t[j], valid[j], kb - WX / 32, KS, g);
  }
};

template <int K>
struct MemB {
  const float* x;
  const int64_t* t;
  const bool* valid;
  int g;
  __device__ __forceinline__ bf16x8 operator()(int kb, int j) const { return ld_frag32(x, K, t[j], valid[j], kb, K, g); }
};

// Register-fed layer computed in NP passes over its RBO output row blocks
// (accumulators for RBO/NP blocks at a time; every weight fragment is still
// loaded once).  epi(rb, j, v) finalises a block in place; with FRAGS the
// finalised values also become the B fragments `out` of the next layer.
constexpr int np_of(int rbo) { return rbo >= 8 ? 2 : 1; }

template <int RBO, int KB, int NP, bool FRAGS, class EPI>
__device__ __forceinline__ void layer_reg(const uint4* __restrict__ W, Stage& S, const bf16x8 (&in)[KB][JW],
                                          bf16x8 (&out)[cdiv(RBO, 2)][JW], EPI epi, int lane, int tid) {
  static_assert(RBO % NP == 0, "passes must split the rows evenly");
  constexpr int RP = RBO / NP;
  static_assert(NP == 1 || RP % 2 == 0, "a pass must hold whole k-blocks of the next layer");
  static_for<0, NP>([&](auto P) __attribute__((always_inline)) {
    constexpr int p = decltype(P)::value;
    f32x4 acc[RP][JW];
    gemm_lds<RP, KB, p * RP>(W, S, RegB<KB>{in}, acc, lane, tid);
#pragma unroll
    for (int rb = 0; rb < RP; ++rb)
#pragma unroll
      for (int j = 0; j < JW; ++j) epi(p * RP + rb, j, acc[rb][j]);
    if constexpr (FRAGS) {
      const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < cdiv(RP, 2); ++kb)
#pragma unroll
        for (int j = 0; j < JW; ++j)
          out[p * RP / 2 + kb][j] = pack8(acc[2 * kb][j], (2 * kb + 1 < RP) ? acc[2 * kb + 1][j] : z);
    }
  });
}

// ---------------------------------------------------------------------------
// kernel arguments

struct ChainArgs {
  RowRange rr;
  const float* geo;
  const int32_t* eidx;
  const int32_t* col;
  const int32_t* species;
  const int64_t* seg;
  int64_t B;
  const double* ges;
  const double* sp_scale;
  double escale;
  int S, nb;
  float r_cut;
  const float* w0;        // first two-body layer, float32 [T0][2S + nb]
  const float* w_eff;     // [W]
  const uint4* tbf[kMaxTwobody];
  const uint4* tbb[kMaxTwobody];
  const uint4* envf;      // environment embedding (forward) used after this MLP
  const uint4* envb;      // transposed environment embedding (adjoint) used before it
  const uint4* latf[kMaxDepth];
  const uint4* latb[kMaxDepth];
  const float* xprev;     // x^{L-1}
  float* xnew;            // x^L (or x^0)
  const float* s;         // s^L
  float* omega;           // omega^{L+1} (or omega^1)
  float* eps;             // edge energies (global edge index)
  uint2* pre[kMaxDepth];  // bf16 pre-activations per MLP layer
  float* gx;              // dE/dx (in: of x^L / x^0; out: of x^{L-1})
  float* gs;              // dE/ds^L
  const float* gomega;    // dE/domega^{L+1} (or of omega^1)
  float* gy;              // [t][16], dE/du at [9]
  float* grho;            // [t][16]
};

struct Cols {
  int64_t t[JW];
  bool valid[JW];
  float u[JW];
};

// Columns of this wavefront's tile.  Returns false (for the whole
// workgroup, uniformly) when the workgroup has no edges; wavefronts past the
// end run with all columns invalid so the workgroup's barriers stay matched.
__device__ __forceinline__ bool tile_cols(const ChainArgs& a, int64_t tile, int lane, int64_t& e0, Cols& c) {
  int64_t e1;
  a.rr.get(e0, e1);
  const int64_t M = e1 - e0;
  if ((int64_t)blockIdx.x * WAVES * TILE >= M) return false;
#pragma unroll
  for (int j = 0; j < JW; ++j) {
    c.t[j] = tile * TILE + 16 * j + (lane & 15);
    c.valid[j] = c.t[j] < M;
    c.u[j] = c.valid[j] ? a.geo[c.t[j] * GEO_STRIDE + GEO_U] : 0.0f;
  }
  return true;
}

#define AFM_CHAIN_PROLOGUE                                                   \
  __shared__ Stage S;                                                        \
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4;               \
  const int64_t tile = (int64_t)blockIdx.x * WAVES + (tid >> 6);             \
  int64_t e0;                                                                \
  Cols c;                                                                    \
  if (!tile_cols(a, tile, lane, e0, c)) return;

// ---------------------------------------------------------------------------
// two-body MLP + environment embedding of layer 1 (forward)

template <int T0, int T1, int T2, int W, int ENV>
__global__ void __launch_bounds__(256) k_tb_fwd(ChainArgs a) {
  AFM_CHAIN_PROLOGUE
  constexpr int NT = T2 ? 3 : 2;
  constexpr int TL = NT == 3 ? T2 : T1;
  static_assert(TL == W, "last two-body width must equal the latent width");
  // first layer on the vector ALUs: gathers of the one-hot columns + rho
  constexpr int RB0 = cdiv(T0, 16);
  bf16x8 in0[cdiv(RB0, 2)][JW];
  {
    f32x4 h0[RB0][JW];
    const int K0 = 2 * a.S + a.nb;
#pragma unroll
    for (int j = 0; j < JW; ++j) {
      float rho[16];
      int zi = 0, zj = 0;
#pragma unroll
      for (int n = 0; n < 16; ++n) rho[n] = 0.0f;
      if (c.valid[j]) {
        const float r = a.geo[c.t[j] * GEO_STRIDE + GEO_D];
        const float pre = sqrtf(2.0f / a.r_cut) / r * c.u[j];
#pragma unroll
        for (int n = 0; n < 16; ++n)
          if (n < a.nb) rho[n] = pre * __sinf((n + 1) * 3.14159265358979323846f * r / a.r_cut);
        zi = min(max(a.species[a.eidx[c.t[j]]], 0), a.S - 1);
        zj = min(max(a.species[a.col[e0 + c.t[j]]], 0), a.S - 1);
      }
#pragma unroll
      for (int rb = 0; rb < RB0; ++rb) {
        f32x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = 16 * rb + 4 * g + q;
          float sacc = 0.0f;
          if (f < T0 && c.valid[j]) {
            const float* w = a.w0 + (int64_t)f * K0;
            sacc = w[zi] + w[a.S + zj];
#pragma unroll
            for (int n = 0; n < 16; ++n)
              if (n < a.nb) sacc += w[2 * a.S + n] * rho[n];
          }
          v[q] = sacc;
        }
        st_pre(a.pre[0], tile, RB0, rb, j, lane, v);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = v[q] * sigm(v[q]);
        h0[rb][j] = v;
      }
    }
    to_frags<RB0>(h0, in0);
  }
  constexpr int RB1 = cdiv(T1, 16);
  constexpr int RBW = W / 16;
  auto silu_epi = [&](uint2* pre, int RB, bool env_out) {
    return [=, &c](int rb, int j, f32x4& v) {
      st_pre(pre, tile, RB, rb, j, lane, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = env_out ? c.u[j] * v[q] * sigm(v[q]) : v[q] * sigm(v[q]);
      if (env_out && c.valid[j]) st4(a.xnew + c.t[j] * W + 16 * rb + 4 * g, v);
    };
  };
  bf16x8 xin[W / 32][JW];
  if constexpr (NT == 3) {
    bf16x8 in1[cdiv(RB1, 2)][JW];
    layer_reg<RB1, cdiv(RB0, 2), 1, true>(a.tbf[1], S, in0, in1, silu_epi(a.pre[1], RB1, false), lane, tid);
    layer_reg<RBW, cdiv(RB1, 2), np_of(RBW), true>(a.tbf[2], S, in1, xin, silu_epi(a.pre[2], RBW, true), lane, tid);
  } else {
    layer_reg<RB1, cdiv(RB0, 2), 1, true>(a.tbf[1], S, in0, xin, silu_epi(a.pre[1], RB1, true), lane, tid);
  }
  // omega^1 = W_env^1 x^0
  constexpr int RBE = ENV / 16;
  bf16x8 unused[cdiv(RBE, 2)][JW];
  layer_reg<RBE, W / 32, np_of(RBE), false>(
      a.envf, S, xin, unused,
      [&](int rb, int j, f32x4& v) {
        if (c.valid[j]) st4(a.omega + c.t[j] * ENV + 16 * rb + 4 * g, v);
      },
      lane, tid);
}

// ---------------------------------------------------------------------------
// latent MLP of one layer (forward) + next environment embedding or energies

template <int W, int KS, int ENV, int DEPTH, bool LAST>
__global__ void __launch_bounds__(256) k_lat_fwd(ChainArgs a) {
  AFM_CHAIN_PROLOGUE
  constexpr int RBW = W / 16, KBW = W / 32;
  constexpr int KIN = W + KS;
  const float r2 = 0.70710678118654752f;
  bf16x8 in[KBW][JW];
  {
    f32x4 h[RBW][JW];
    gemm_lds<RBW, cdiv(KIN, 32), 0>(a.latf[0], S, CatB<W, KS>{a.xprev, a.s, c.t, c.valid, g}, h, lane, tid);
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        st_pre(a.pre[0], tile, RBW, rb, j, lane, h[rb][j]);
        if (DEPTH > 1) {
#pragma unroll
          for (int q = 0; q < 4; ++q) h[rb][j][q] = h[rb][j][q] * sigm(h[rb][j][q]);
        } else {
          const f32x4 xp = c.valid[j] ? ld4(a.xprev + c.t[j] * W + 16 * rb + 4 * g) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < 4; ++q) h[rb][j][q] = (xp[q] + c.u[j] * h[rb][j][q] * sigm(h[rb][j][q])) * r2;
          if (!LAST && c.valid[j]) st4(a.xnew + c.t[j] * W + 16 * rb + 4 * g, h[rb][j]);
        }
      }
    to_frags<RBW>(h, in);
  }
  float ep[JW];
#pragma unroll
  for (int j = 0; j < JW; ++j) ep[j] = 0.0f;
  static_for<1, DEPTH>([&](auto K) __attribute__((always_inline)) {
    constexpr int k = decltype(K)::value;
    constexpr bool last = k == DEPTH - 1;
    bf16x8 out[KBW][JW];
    layer_reg<RBW, KBW, np_of(RBW), true>(
        a.latf[k], S, in, out,
        [&](int rb, int j, f32x4& v) {
          st_pre(a.pre[k], tile, RBW, rb, j, lane, v);
          if constexpr (!last) {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = v[q] * sigm(v[q]);
          } else {
            const f32x4 xp = c.valid[j] ? ld4(a.xprev + c.t[j] * W + 16 * rb + 4 * g) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = (xp[q] + c.u[j] * v[q] * sigm(v[q])) * r2;
            if constexpr (!LAST) {
              if (c.valid[j]) st4(a.xnew + c.t[j] * W + 16 * rb + 4 * g, v);
            } else {
              const f32x4 we = ld4(a.w_eff + 16 * rb + 4 * g);
#pragma unroll
              for (int q = 0; q < 4; ++q) ep[j] += we[q] * v[q];
            }
          }
        },
        lane, tid);
#pragma unroll
    for (int kb = 0; kb < KBW; ++kb)
#pragma unroll
      for (int j = 0; j < JW; ++j) in[kb][j] = out[kb][j];
  });
  if constexpr (!LAST) {
    constexpr int RBE = ENV / 16;
    bf16x8 unused[cdiv(RBE, 2)][JW];
    layer_reg<RBE, KBW, np_of(RBE), false>(
        a.envf, S, in, unused,
        [&](int rb, int j, f32x4& v) {
          if (c.valid[j]) st4(a.omega + c.t[j] * ENV + 16 * rb + 4 * g, v);
        },
        lane, tid);
  } else {
    // eps_e = w_eff . x^{N_L}
#pragma unroll
    for (int j = 0; j < JW; ++j) {
      float p = ep[j];
      p += __shfl_xor(p, 16, 64);
      p += __shfl_xor(p, 32, 64);
      if (g == 0 && c.valid[j]) a.eps[e0 + c.t[j]] = p;
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint of one latent layer: dE/dx^L -> dE/dx^{L-1}, dE/ds^L, dE/du

template <int W, int KS, int ENV, int DEPTH, bool LAST>
__global__ void __launch_bounds__(256) k_lat_bwd(ChainArgs a) {
  AFM_CHAIN_PROLOGUE
  constexpr int RBW = W / 16, KBW = W / 32;
  const float r2 = 0.70710678118654752f;
  bf16x8 in[KBW][JW];
  {
    f32x4 G[RBW][JW];
    if constexpr (LAST) {
      // dE/dx^{N_L} = sigma_Z(i) escale gE_s w_eff
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        float ce = 0.0f;
        if (c.valid[j]) {
          const int64_t i = a.eidx[c.t[j]];
          ce = (float)(a.sp_scale[min(max(a.species[i], 0), a.S - 1)] * a.escale);
          if (a.ges) {
            int64_t lo = 0, hi = a.B;
            while (hi - lo > 1) {
              int64_t mid = (lo + hi) >> 1;
              if (a.seg[mid] <= i) lo = mid; else hi = mid;
            }
            ce *= (float)a.ges[lo];
          }
        }
#pragma unroll
        for (int rb = 0; rb < RBW; ++rb) {
          const f32x4 we = ld4(a.w_eff + 16 * rb + 4 * g);
#pragma unroll
          for (int q = 0; q < 4; ++q) G[rb][j][q] = ce * we[q];
        }
      }
    } else {
      // dE/dx^L = (stored) + W_env^{L+1 T} dE/domega^{L+1}
      gemm_lds<RBW, cdiv(ENV, 32), 0>(a.envb, S, MemB<ENV>{a.gomega, c.t, c.valid, g}, G, lane, tid);
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int j = 0; j < JW; ++j)
          if (c.valid[j]) G[rb][j] += ld4(a.gx + c.t[j] * W + 16 * rb + 4 * g);
    }
    // head: x^L = (x^{L-1} + u silu(a_D)) / sqrt 2
    float gu[JW];
#pragma unroll
    for (int j = 0; j < JW; ++j) gu[j] = 0.0f;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        const f32x4 pa = ld_pre(a.pre[DEPTH - 1], tile, RBW, rb, j, lane);
        f32x4 res;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float gs_ = G[rb][j][q] * r2;
          const float sg = sigm(pa[q]);
          res[q] = gs_;
          gu[j] += gs_ * pa[q] * sg;
          G[rb][j][q] = gs_ * c.u[j] * sg * (1.0f + pa[q] * (1.0f - sg));
        }
        if (c.valid[j]) st4(a.gx + c.t[j] * W + 16 * rb + 4 * g, res);
      }
#pragma unroll
    for (int j = 0; j < JW; ++j) {
      float v = gu[j];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (g == 0 && c.valid[j]) a.gy[c.t[j] * GEO_STRIDE + 9] += v;
    }
    to_frags<RBW>(G, in);
  }
  // inner layers: ga_{k-1} = (W_k^T ga_k) * silu'(a_{k-1})
  static_for<1, DEPTH>([&](auto KK) __attribute__((always_inline)) {
    constexpr int k = DEPTH - decltype(KK)::value;
    bf16x8 out[KBW][JW];
    layer_reg<RBW, KBW, np_of(RBW), true>(
        a.latb[k], S, in, out,
        [&](int rb, int j, f32x4& v) {
          const f32x4 pa = ld_pre(a.pre[k - 1], tile, RBW, rb, j, lane);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float sg = sigm(pa[q]);
            v[q] *= sg * (1.0f + pa[q] * (1.0f - sg));
          }
        },
        lane, tid);
#pragma unroll
    for (int kb = 0; kb < KBW; ++kb)
#pragma unroll
      for (int j = 0; j < JW; ++j) in[kb][j] = out[kb][j];
  });
  // dE/d[x | s] = W_1^T ga_1: x rows added to the residual share, s rows stored
  {
    bf16x8 unused[KBW][JW];
    layer_reg<RBW, KBW, np_of(RBW), false>(
        a.latb[0], S, in, unused,
        [&](int rb, int j, f32x4& v) {
          if (c.valid[j]) {
            float* p = a.gx + c.t[j] * W + 16 * rb + 4 * g;
            st4(p, ld4(p) + v);
          }
        },
        lane, tid);
  }
  {
    constexpr int RBS = KS / 16;
    f32x4 os[RBS][JW];
    gemm_lds<RBS, KBW, RBW>(a.latb[0], S, RegB<KBW>{in}, os, lane, tid);
#pragma unroll
    for (int rb = 0; rb < RBS; ++rb)
#pragma unroll
      for (int j = 0; j < JW; ++j)
        if (c.valid[j]) st4(a.gs + c.t[j] * KS + 16 * rb + 4 * g, os[rb][j]);
  }
}

// ---------------------------------------------------------------------------
// adjoint of the two-body MLP: dE/dx^0 (+ W_env^1T dE/domega^1) -> dE/drho, dE/du

template <int T0, int T1, int T2, int W, int ENV>
__global__ void __launch_bounds__(256) k_tb_bwd(ChainArgs a) {
  AFM_CHAIN_PROLOGUE
  constexpr int NT = T2 ? 3 : 2;
  constexpr int RBW = W / 16;
  constexpr int RB0 = cdiv(T0, 16), RB1 = cdiv(T1, 16);
  bf16x8 in[RBW / 2][JW];
  {
    f32x4 G[RBW][JW];
    gemm_lds<RBW, cdiv(ENV, 32), 0>(a.envb, S, MemB<ENV>{a.gomega, c.t, c.valid, g}, G, lane, tid);
    // head: x^0 = u silu(a_last)
    float gu[JW];
#pragma unroll
    for (int j = 0; j < JW; ++j) gu[j] = 0.0f;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        const f32x4 gx = c.valid[j] ? ld4(a.gx + c.t[j] * W + 16 * rb + 4 * g) : f32x4{0.f, 0.f, 0.f, 0.f};
        const f32x4 pa = ld_pre(a.pre[NT - 1], tile, RBW, rb, j, lane);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float gv = G[rb][j][q] + gx[q];
          const float sg = sigm(pa[q]);
          gu[j] += gv * pa[q] * sg;
          G[rb][j][q] = gv * c.u[j] * sg * (1.0f + pa[q] * (1.0f - sg));
        }
      }
#pragma unroll
    for (int j = 0; j < JW; ++j) {
      float v = gu[j];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (g == 0 && c.valid[j]) a.gy[c.t[j] * GEO_STRIDE + 9] += v;
    }
    to_frags<RBW>(G, in);
  }
  auto dsilu_epi = [&](uint2* pre, int RB) {
    return [=](int rb, int j, f32x4& v) {
      const f32x4 pa = ld_pre(pre, tile, RB, rb, j, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float sg = sigm(pa[q]);
        v[q] *= sg * (1.0f + pa[q] * (1.0f - sg));
      }
    };
  };
  bf16x8 in1[cdiv(RB1, 2)][JW];
  if constexpr (NT == 3) {
    layer_reg<RB1, RBW / 2, np_of(RB1), true>(a.tbb[2], S, in, in1, dsilu_epi(a.pre[1], RB1), lane,
                                                          tid);
  } else {
#pragma unroll
    for (int kb = 0; kb < cdiv(RB1, 2); ++kb)
#pragma unroll
      for (int j = 0; j < JW; ++j) in1[kb][j] = in[kb][j];
  }
  f32x4 G0[RB0][JW];
  gemm_lds<RB0, cdiv(RB1, 2), 0>(a.tbb[1], S, RegB<cdiv(RB1, 2)>{in1}, G0, lane, tid);
#pragma unroll
  for (int rb = 0; rb < RB0; ++rb)
#pragma unroll
    for (int j = 0; j < JW; ++j) {
      const f32x4 pa = ld_pre(a.pre[0], tile, RB0, rb, j, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float sg = sigm(pa[q]);
        G0[rb][j][q] *= sg * (1.0f + pa[q] * (1.0f - sg));
      }
    }
  // dE/drho_n = sum_f W_0[f][2S + n] ga_0[f]
  const int K0 = 2 * a.S + a.nb;
#pragma unroll
  for (int j = 0; j < JW; ++j) {
    for (int n = 0; n < a.nb; ++n) {
      float p = 0.0f;
#pragma unroll
      for (int rb = 0; rb < RB0; ++rb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = 16 * rb + 4 * g + q;
          if (f < T0) p += a.w0[(int64_t)f * K0 + 2 * a.S + n] * G0[rb][j][q];
        }
      p += __shfl_xor(p, 16, 64);
      p += __shfl_xor(p, 32, 64);
      if (g == 0 && c.valid[j]) a.grho[c.t[j] * 16 + n] = p;
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch over the built shapes: (w, c, l_max, depth, two-body widths, n0e)

#define AFM_SHAPES(X)                       \
  X(32, 8, 1, 2, 16, 32, 0, 2)              \
  X(64, 16, 2, 3, 16, 32, 64, 3)            \
  X(128, 32, 2, 3, 32, 64, 128, 3)          \
  X(256, 64, 2, 3, 64, 128, 256, 3)

static bool shape_is(const ModelDims& d, int w, int c, int lmax, int depth, int t0, int t1, int t2, int n0e) {
  if (d.w != w || d.c != c || d.lmax != lmax || d.depth != depth) return false;
  if (t2 ? (d.ntb != 3 || d.tb[0] != t0 || d.tb[1] != t1 || d.tb[2] != t2)
         : (d.ntb != 2 || d.tb[0] != t0 || d.tb[1] != t1))
    return false;
  const Plan P = make_plan(d.lmax, d.NL);
  for (int L = 0; L < d.NL; ++L)
    if (P.layer[L].n0e != n0e) return false;
  return d.nb <= 16;
}

int mfma_check_shape(const afm_model* m) {
#define X(w, c, l, dp, a0, a1, a2, n0) \
  if (shape_is(m->dims, w, c, l, dp, a0, a1, a2, n0)) return AFM_OK;
  AFM_SHAPES(X)
#undef X
  set_error("BF16 MFMA kernels are built for (w, c, l_max, depth, two-body) = (32,8,1,2,[16,32]), "
            "(64,16,2,3,[16,32,64]), (128,32,2,3,[32,64,128]), (256,64,2,3,[64,128,256])");
  return AFM_E_UNSUPPORTED;
}

static ChainArgs base_args(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                           const int32_t* species) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  const char* fb = static_cast<const char*>(m->W.frag);
  ChainArgs a{};
  a.rr = rr;
  a.geo = ws_ptr<float>(ws, L.geo);
  a.eidx = ws_ptr<int32_t>(ws, L.eidx);
  a.species = species;
  a.sp_scale = m->W.sp_scale;
  a.escale = d.escale;
  a.S = d.S;
  a.nb = d.nb;
  a.r_cut = (float)d.r_cut;
  a.w0 = m->W.tb[0];
  a.w_eff = m->W.w_eff;
  for (int k = 1; k < d.ntb; ++k) {
    a.tbf[k] = reinterpret_cast<const uint4*>(fb + fo->tbf[k]);
    a.tbb[k] = reinterpret_cast<const uint4*>(fb + fo->tbb[k]);
  }
  a.gy = ws_ptr<float>(ws, L.gy);
  a.grho = ws_ptr<float>(ws, L.grho);
  a.gx = ws_ptr<float>(ws, L.gx);
  a.gs = ws_ptr<float>(ws, L.gs);
  a.gomega = ws_ptr<float>(ws, L.gomega);
  return a;
}

static const uint4* frag_ptr(const afm_model* m, int64_t off) {
  return reinterpret_cast<const uint4*>(static_cast<const char*>(m->W.frag) + off);
}

static dim3 chain_grid(const WsLayout& L) { return dim3(grid_for(L.cex, TILE * WAVES)); }

int mfma_twobody_fwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                     const int32_t* species, const int32_t* col, hipStream_t st) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, species);
  a.col = col;
  a.envf = frag_ptr(m, fo->envf[0]);
  a.xnew = ws_ptr<float>(ws, L.x[0]);
  a.omega = ws_ptr<float>(ws, L.omega[0]);
  for (int k = 0; k < d.ntb; ++k) a.pre[k] = ws_ptr<uint2>(ws, L.tb_pre[k]);
#define X(w, c, l, dp, a0, a1, a2, n0)                                                             \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                  \
    hipLaunchKernelGGL((k_tb_fwd<a0, a1, a2, w, (l + 1) * c>), chain_grid(L), dim3(256), 0, st, a); \
    AFM_LAUNCH_CHECK();                                                                            \
    return AFM_OK;                                                                                 \
  }
  AFM_SHAPES(X)
#undef X
  return mfma_check_shape(m);
}

int mfma_twobody_bwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                     const int32_t* species, hipStream_t st) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, species);
  a.envb = frag_ptr(m, fo->envb[0]);
  for (int k = 0; k < d.ntb; ++k) a.pre[k] = ws_ptr<uint2>(ws, L.tb_pre[k]);
#define X(w, c, l, dp, a0, a1, a2, n0)                                                             \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                  \
    hipLaunchKernelGGL((k_tb_bwd<a0, a1, a2, w, (l + 1) * c>), chain_grid(L), dim3(256), 0, st, a); \
    AFM_LAUNCH_CHECK();                                                                            \
    return AFM_OK;                                                                                 \
  }
  AFM_SHAPES(X)
#undef X
  return mfma_check_shape(m);
}

int mfma_latent_fwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer,
                    hipStream_t st) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, nullptr);
  for (int k = 0; k < d.depth; ++k) a.latf[k] = frag_ptr(m, fo->latf[layer - 1][k]);
  if (layer < d.NL) a.envf = frag_ptr(m, fo->envf[layer]);
  a.xprev = ws_ptr<float>(ws, L.x[layer - 1]);
  a.xnew = layer < d.NL ? ws_ptr<float>(ws, L.x[layer]) : nullptr;
  a.s = ws_ptr<float>(ws, L.s[layer - 1]);
  a.omega = layer < d.NL ? ws_ptr<float>(ws, L.omega[layer]) : nullptr;
  a.eps = ws_ptr<float>(ws, L.eps);
  for (int k = 0; k < d.depth; ++k) a.pre[k] = ws_ptr<uint2>(ws, L.lat_pre[layer - 1][k]);
  const bool last = layer == d.NL;
#define X(w, c, l, dp, a0, a1, a2, n0)                                                                  \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                       \
    if (last)                                                                                           \
      hipLaunchKernelGGL((k_lat_fwd<w, n0 * c, (l + 1) * c, dp, true>), chain_grid(L), dim3(256), 0, st, a);  \
    else                                                                                                \
      hipLaunchKernelGGL((k_lat_fwd<w, n0 * c, (l + 1) * c, dp, false>), chain_grid(L), dim3(256), 0, st, a); \
    AFM_LAUNCH_CHECK();                                                                                 \
    return AFM_OK;                                                                                      \
  }
  AFM_SHAPES(X)
#undef X
  return mfma_check_shape(m);
}

int mfma_latent_bwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer,
                    const int32_t* species, const int64_t* seg, int64_t B, const double* grad_e_struct,
                    hipStream_t st) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, species);
  a.seg = seg;
  a.B = B;
  a.ges = grad_e_struct;
  for (int k = 0; k < d.depth; ++k) a.latb[k] = frag_ptr(m, fo->latb[layer - 1][k]);
  if (layer < d.NL) a.envb = frag_ptr(m, fo->envb[layer]);
  for (int k = 0; k < d.depth; ++k) a.pre[k] = ws_ptr<uint2>(ws, L.lat_pre[layer - 1][k]);
  const bool last = layer == d.NL;
#define X(w, c, l, dp, a0, a1, a2, n0)                                                                  \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                       \
    if (last)                                                                                           \
      hipLaunchKernelGGL((k_lat_bwd<w, n0 * c, (l + 1) * c, dp, true>), chain_grid(L), dim3(256), 0, st, a);  \
    else                                                                                                \
      hipLaunchKernelGGL((k_lat_bwd<w, n0 * c, (l + 1) * c, dp, false>), chain_grid(L), dim3(256), 0, st, a); \
    AFM_LAUNCH_CHECK();                                                                                 \
    return AFM_OK;                                                                                      \
  }
  AFM_SHAPES(X)
#undef X
  return mfma_check_shape(m);
}

}  // namespace afm
