// Kernels and launchers of the BF16 MFMA chains for one edge-tile shape.
// Included by mfma_chain.hip once per tile shape, inside a namespace that
// defines NCB (16-edge column blocks per workgroup tile), NCBW (column
// blocks per wavefront) and WPE (wavefronts per SIMD the kernels are
// compiled for); everything here depends on them.  A workgroup of
// NPS x NCB / NCBW wavefronts owns a tile of TILE = 16 NCB edges: 8 pair
// slots times NCB / NCBW column groups of 16 NCBW edges.

constexpr int TILE = 16 * NCB;    // edges per workgroup
constexpr int NPS = 8;            // output-row pair slots per workgroup
constexpr int NWAVE = NPS * (NCB / NCBW);  // wavefronts: pair slot x column group
constexpr int NTHR = 64 * NWAVE;
static_assert(NCB % NCBW == 0, "whole column groups");

// Latent widths above 256 (more output-row pairs than pair slots) give each
// wavefront NPP pairs, pslot + j NPS; their LDS tiles leave one workgroup
// per CU, so those kernels are compiled for 2 wavefronts per SIMD.
template <int W>
constexpr int wpe_for() { return W > 256 ? 2 : WPE; }

// ---------------------------------------------------------------------------
// device building blocks

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sigm(float a) { return __builtin_amdgcn_rcpf(1.0f + __expf(-a)); }
// silu'(a) = s (1 + a (1 - s)), s = sigmoid(a)
__device__ __forceinline__ float dsilu_of(float a) {
  const float sg = sigm(a);
  return sg * (1.0f + a * (1.0f - sg));
}

__device__ __forceinline__ bf16x8 pack8(f32x4 lo, f32x4 hi) {
  bf16x8 r;
  r[0] = (__bf16)lo[0]; r[1] = (__bf16)lo[1]; r[2] = (__bf16)lo[2]; r[3] = (__bf16)lo[3];
  r[4] = (__bf16)hi[0]; r[5] = (__bf16)hi[1]; r[6] = (__bf16)hi[2]; r[7] = (__bf16)hi[3];
  return r;
}

// v - bf16(v) rounded to bf16 again, for the values packed in `hi`: the
// second term of a two-term bf16 representation (~16 mantissa bits)
__device__ __forceinline__ bf16x8 pack_rem(f32x4 lo, f32x4 hi, bf16x8 h) {
  bf16x8 r;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    r[q] = (__bf16)(lo[q] - (float)h[q]);
    r[4 + q] = (__bf16)(hi[q] - (float)h[4 + q]);
  }
  return r;
}

__device__ __forceinline__ f32x4 ld4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }
__device__ __forceinline__ void st4(float* p, f32x4 v) { *reinterpret_cast<f32x4*>(p) = v; }
// The forward's per-edge outputs (x^L, omega, pre-activations) are read
// only by later kernels, after other large streams: streaming
// (non-temporal) stores, so that they do not displace the weight fragments
// every tile re-reads from L2.  The adjoint's outputs, read by the very next
// kernel, use plain stores.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st4_stream(float* p, f32x4 v) {
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p));
}
__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// pre-activation tile storage: [tile][RB][NCB][64 lanes][4] bf16 (streamed)
__device__ __forceinline__ void st_pre(uint2* pre, int64_t tile, int RB, int rb, int cb, int lane, f32x4 v) {
  bf16x4 h;
  h[0] = (__bf16)v[0]; h[1] = (__bf16)v[1]; h[2] = (__bf16)v[2]; h[3] = (__bf16)v[3];
  __builtin_nontemporal_store(__builtin_bit_cast(u32x2, h),
                              reinterpret_cast<u32x2*>(pre + ((tile * RB + rb) * NCB + cb) * 64 + lane));
}
__device__ __forceinline__ f32x4 ld_pre(const uint2* pre, int64_t tile, int RB, int rb, int cb, int lane) {
  const bf16x4 h = __builtin_bit_cast(bf16x4, pre[((tile * RB + rb) * NCB + cb) * 64 + lane]);
  f32x4 v;
  v[0] = (float)h[0]; v[1] = (float)h[1]; v[2] = (float)h[2]; v[3] = (float)h[3];
  return v;
}

// LDS: two activation buffers of B fragments [kb][cb][64 lanes] (bf16 x 8
// each) and a [pair slot][edge] scratch row for cross-wavefront sums
template <int KMAX>
struct ChainSmem {
  uint4 act[2][cdiv(KMAX, 32) * NCB * 64];
  float red[NPS][TILE];
};
__device__ __forceinline__ int frag_idx(int kb, int cb, int lane) { return (kb * NCB + cb) * 64 + lane; }

// B fragment of features [32 kb, 32 kb + 32) of row t of a float32
// row-major matrix X[t][K] (zeros beyond K and for invalid rows)
template <int K>
__device__ __forceinline__ bf16x8 ld_frag32(const float* __restrict__ X, int64_t t, bool valid, int kb, int g) {
  const int fa = 32 * kb + 4 * g, fb = fa + 16;
  const f32x4 lo = (valid && fa + 4 <= K) ? ld4(X + t * K + fa) : zero4();
  const f32x4 hi = (valid && fb + 4 <= K) ? ld4(X + t * K + fb) : zero4();
  return pack8(lo, hi);
}

// Staging of tile rows [tile*TILE, tile*TILE + TILE) of a row-major matrix
// X[t][K] into LDS B fragments.  A stager issues all of a thread's global
// loads (load) before the first LDS write (store), so a tile costs one
// memory round trip, not one per fragment; rows past the chunk load row
// tile*TILE (always valid) and are zeroed.  F32 = true: float32 source
// (rounded to bf16), false: bf16 source (8-byte words copied).
template <int K, bool F32>
struct Stager {
  static constexpr int NF = cdiv(K, 32) * NCB * 64;
  static constexpr int IT = cdiv(NF, NTHR);
  typedef typename std::conditional<F32, f32x4, uint2>::type V;
  V lo[IT], hi[IT];
  __device__ __forceinline__ void load(const void* __restrict__ Xv, int64_t tile, int64_t M, int tid) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = tid + it * NTHR;
      const int l = idx & 63, cb = (idx >> 6) % NCB, kb = idx / (64 * NCB);
      const int64_t t = tile * TILE + 16 * cb + (l & 15);
      const int fa = 32 * kb + 4 * (l >> 4), fb = fa + 16;
      const bool valid = idx < NF && t < M;
      const int64_t tr = valid ? t : tile * TILE;
      if constexpr (F32) {
        const float* X = static_cast<const float*>(Xv) + tr * K;
        lo[it] = (K % 32 == 0 || fa + 4 <= K) ? ld4(X + fa) : zero4();
        hi[it] = (K % 32 == 0 || fb + 4 <= K) ? ld4(X + fb) : zero4();
        if (!valid) { lo[it] = zero4(); hi[it] = zero4(); }
      } else {
        const uint16_t* X = static_cast<const uint16_t*>(Xv) + tr * K;
        lo[it] = (K % 32 == 0 || fa + 4 <= K) ? *reinterpret_cast<const uint2*>(X + fa) : uint2{0u, 0u};
        hi[it] = (K % 32 == 0 || fb + 4 <= K) ? *reinterpret_cast<const uint2*>(X + fb) : uint2{0u, 0u};
        if (!valid) { lo[it] = uint2{0u, 0u}; hi[it] = uint2{0u, 0u}; }
      }
    }
  }
  __device__ __forceinline__ void store(uint4* __restrict__ act, int tid) const {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = tid + it * NTHR;
      if (NF % NTHR == 0 || idx < NF) {
        if constexpr (F32) act[idx] = __builtin_bit_cast(uint4, pack8(lo[it], hi[it]));
        else act[idx] = uint4{lo[it].x, lo[it].y, hi[it].x, hi[it].y};
      }
    }
  }
};

template <int K>
__device__ __forceinline__ void stage_rows(uint4* __restrict__ act, const float* __restrict__ X, int64_t tile,
                                           int64_t M, int tid) {
  Stager<K, true> s;
  s.load(X, tile, M, tid);
  s.store(act, tid);
}

template <int K>
__device__ __forceinline__ void stage_rows_bf16(uint4* __restrict__ act, const uint16_t* __restrict__ X,
                                                int64_t tile, int64_t M, int tid) {
  Stager<K, false> s;
  s.load(X, tile, M, tid);
  s.store(act, tid);
}

// The same one fragment at a time (few registers; for a restage of rows
// the tile has just read, which hit in L2)
template <int K>
__device__ __forceinline__ void restage_rows_bf16(uint4* __restrict__ act, const uint16_t* __restrict__ X,
                                                  int64_t tile, int64_t M, int tid) {
  constexpr int NF = cdiv(K, 32) * NCB * 64;
#pragma unroll 1
  for (int idx = tid; idx < NF; idx += NTHR) {
    const int l = idx & 63, cb = (idx >> 6) % NCB, kb = idx / (64 * NCB), g = l >> 4;
    const int64_t t = tile * TILE + 16 * cb + (l & 15);
    const int fa = 32 * kb + 4 * g, fb = fa + 16;
    const bool valid = t < M;
    const uint2 lo = (valid && fa + 4 <= K) ? *reinterpret_cast<const uint2*>(X + t * K + fa) : uint2{0u, 0u};
    const uint2 hi = (valid && fb + 4 <= K) ? *reinterpret_cast<const uint2*>(X + t * K + fb) : uint2{0u, 0u};
    act[idx] = uint4{lo.x, lo.y, hi.x, hi.y};
  }
}

// four consecutive bf16 values (8-byte streaming store)
__device__ __forceinline__ void st_bf16x4(uint16_t* p, f32x4 v) {
  const uint4 w = __builtin_bit_cast(uint4, pack8(v, v));
  __builtin_nontemporal_store(u32x2{w.x, w.y}, reinterpret_cast<u32x2*>(p));
}
// the same with a plain store (for outputs the next kernel reads at once)
__device__ __forceinline__ void st_bf16x4_plain(uint16_t* p, f32x4 v) {
  const uint4 w = __builtin_bit_cast(uint4, pack8(v, v));
  *reinterpret_cast<u32x2*>(p) = u32x2{w.x, w.y};
}

// acc[r][cb] += sum over k-blocks kb in [kb0, kb0 + NKB) of
//   W[2 pair + r][kb] x act[kb - kb0][cb]
// W: packed weight fragments [RB][KBW][hi, lo][64]; act: LDS fragments.
// NS = 2 uses w = hi + lo, NS = 1 the hi term alone (the lo fragments are
// then never loaded).  Weight fragments stream from L2 one k-block ahead;
// per k-block the hi products of both row blocks and all column blocks are
// issued before the lo products, so the two MFMAs into one accumulator are
// 16 apart.
// KLO > 0: the input activations are carried as two bf16 terms too (b =
// b_hi + b_lo, the lo fragments KLO k-blocks after the hi ones), and each
// product adds W_hi x b_lo to W_hi x b_hi + W_lo x b_hi (the W_lo x b_lo term,
// ~2^-16 of the product, is dropped).
template <int KBW, int NKB, int NS = kSplit, int KLO = 0>
__device__ __forceinline__ void mma_pair(const uint4* __restrict__ W, int pair, int kb0, const uint4* act,
                                         f32x4 (&acc)[2][NCBW], int half, int lane) {
  static_assert(NS == 1 || NS == kSplit, "NS");
  const uint4* w0 = W + ((int64_t)(2 * pair) * KBW + kb0) * (kSplit * 64) + lane;
  const uint4* w1 = w0 + (int64_t)KBW * (kSplit * 64);
  uint4 cur[2][NS], nxt[2][NS];
#pragma unroll
  for (int h = 0; h < NS; ++h) {
    cur[0][h] = w0[64 * h];
    cur[1][h] = w1[64 * h];
  }
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    if (kb + 1 < NKB) {
      const int o = (kb + 1) * (kSplit * 64);
#pragma unroll
      for (int h = 0; h < NS; ++h) {
        nxt[0][h] = w0[o + 64 * h];
        nxt[1][h] = w1[o + 64 * h];
      }
    }
    bf16x8 b[NCBW], blo[KLO > 0 ? NCBW : 1];
#pragma unroll
    for (int c = 0; c < NCBW; ++c)
      b[c] = __builtin_bit_cast(bf16x8, act[frag_idx(kb, half * NCBW + c, lane)]);
    if constexpr (KLO > 0) {
#pragma unroll
      for (int c = 0; c < NCBW; ++c)
        blo[c] = __builtin_bit_cast(bf16x8, act[frag_idx(kb + KLO, half * NCBW + c, lane)]);
    }
    // the next k-block's weight loads go out before this block's MFMAs (a
    // whole block of MFMAs covers their L2 latency), not sunk among them
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int h = 0; h < NS; ++h)
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const bf16x8 A = __builtin_bit_cast(bf16x8, cur[r][h]);
#pragma unroll
        for (int c = 0; c < NCBW; ++c) acc[r][c] = mfma(A, b[c], acc[r][c]);
      }
    if constexpr (KLO > 0) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const bf16x8 A = __builtin_bit_cast(bf16x8, cur[r][0]);
#pragma unroll
        for (int c = 0; c < NCBW; ++c) acc[r][c] = mfma(A, blo[c], acc[r][c]);
      }
    }
    if (kb + 1 < NKB) {
#pragma unroll
      for (int h = 0; h < NS; ++h) {
        cur[0][h] = nxt[0][h];
        cur[1][h] = nxt[1][h];
      }
    }
    // keep the scheduler from hoisting later k-blocks' loads (register
    // pressure at 4 wavefronts per SIMD)
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ void zero_acc(f32x4 (&acc)[2][NCBW]) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < NCBW; ++c) acc[r][c] = zero4();
}

// Finalise a pair of row blocks: epi(rb, c, v) in place for both blocks (c
// indexes this wavefront's column blocks), then (if out) the pair becomes
// k-block `pair` of the next layer's input.
template <class EPI>
__device__ __forceinline__ void finish_pair(int pair, f32x4 (&acc)[2][NCBW], uint4* out, EPI&& epi, int half,
                                            int lane, int klo = 0) {
#pragma unroll
  for (int c = 0; c < NCBW; ++c) {
    epi(2 * pair, c, acc[0][c]);
    epi(2 * pair + 1, c, acc[1][c]);
    if (out) {
      const bf16x8 hi = pack8(acc[0][c], acc[1][c]);
      out[frag_idx(pair, half * NCBW + c, lane)] = __builtin_bit_cast(uint4, hi);
      // klo > 0: also the remainder v - bf16(v), klo k-blocks further on
      if (klo) out[frag_idx(pair + klo, half * NCBW + c, lane)] = __builtin_bit_cast(uint4, pack_rem(acc[0][c], acc[1][c], hi));
    }
  }
}

// A whole layer from LDS: rows of NPAIR pairs, the wavefronts of pair slot
// ps own pairs ps, ps + NPS, ...; no barrier inside.
// KLO_IN > 0: the input carries bf16 remainders KLO_IN k-blocks after its
// leading terms; KLO_OUT > 0: so does the output (for the next such layer).
template <int NPAIR, int KBW, int NS = kSplit, int KLO_IN = 0, int KLO_OUT = 0, class EPI>
__device__ __forceinline__ void layer_lds(const uint4* __restrict__ W, const uint4* in, uint4* out, EPI&& epi,
                                          int pslot, int half, int lane) {
  static_for<0, cdiv(NPAIR, NPS)>([&](auto P) __attribute__((always_inline)) {
    const int pair = decltype(P)::value * NPS + pslot;
    if (pair < NPAIR) {
      f32x4 acc[2][NCBW];
      zero_acc(acc);
      mma_pair<KBW, KBW, NS, KLO_IN>(W, pair, 0, in, acc, half, lane);
      finish_pair(pair, acc, out, epi, half, lane, KLO_OUT);
    }
  });
}

// Sum of v over the lane groups g (the 4 row quarters of a C block); the
// result is valid in every lane.
__device__ __forceinline__ float sum_groups(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}


// Workgroup prologue: tile, edge count of the chunk, this lane's envelope
// factor per column block.  The whole workgroup returns when its tile is
// empty (uniform, before any barrier).
#define AFM_TILE_PROLOGUE                                                          \
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4;    \
  const int pslot = wave % NPS, half = wave / NPS;                                 \
  int64_t e0, e1;                                                                  \
  a.rr.get(e0, e1);                                                                \
  const int64_t M = e1 - e0;                                                       \
  const int64_t tile = blockIdx.x;                                                 \
  if (tile * TILE >= M) return;                                                    \
  auto cbA = [&](int c) { return half * NCBW + c; };                               \
  auto col_t = [&](int c) { return tile * TILE + 16 * cbA(c) + (lane & 15); };     \
  float u[NCBW];                                                                   \
  _Pragma("unroll") for (int c = 0; c < NCBW; ++c) {                               \
    const int64_t t = col_t(c);                                                    \
    u[c] = t < M ? a.geo[t * GEO_STRIDE + GEO_U] : 0.0f;                           \
  }

// Per-edge sums of this wavefront's partials part[c] (lane groups already
// summed) over the pair slots; fn(t, total) runs once per valid edge.
template <class FN>
__device__ __forceinline__ void wg_edge_sum(float (&red)[NPS][TILE], const float (&part)[NCBW], int64_t tile,
                                            int64_t M, int tid, FN&& fn) {
  const int lane = tid & 63, wave = tid >> 6, pslot = wave % NPS, half = wave / NPS;
  if ((lane >> 4) == 0) {
#pragma unroll
    for (int c = 0; c < NCBW; ++c) red[pslot][16 * (half * NCBW + c) + lane] = part[c];
  }
  __syncthreads();
  if (tid < TILE) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < NPS; ++w) s += red[w][tid];
    const int64_t t = tile * TILE + tid;
    if (t < M) fn(t, s);
  }
  __syncthreads();
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// ---------------------------------------------------------------------------
// two-body MLP + environment embedding of layer 1 (forward)

template <int T0, int T1, int T2, int W, int ENV>
__global__ void __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(wpe_for<W>()))) k_tb_fwd(ChainArgs a) {
  AFM_TILE_PROLOGUE
  constexpr int NT = T2 ? 3 : 2;
  constexpr int TL = NT == 3 ? T2 : T1;
  static_assert(TL == W, "last two-body width must equal the latent width");
  // The hidden activations of the two-body MLP enter its MFMA layers as two
  // bf16 terms (hi + remainder, ~16 mantissa bits; the remainders KB0 / KB1
  // k-blocks after the leading terms): edges with the same species pair and
  // similar lengths have nearly equal activations here, so single-bf16
  // rounding errors would be correlated across a row and add up in E_i (an
  // FP64 emulation of the rounding put 85 % of the per-atom energy error of
  // the uneven 89-species batch at these two inputs).
  constexpr int KB0 = cdiv(T0, 32), KB1 = cdiv(T1, 32);
  __shared__ ChainSmem<cmax(cmax(64 * KB0, NT == 3 ? 64 * KB1 : 32 * KB1), W)> S;
  constexpr int RB0 = cdiv(T0, 16), RB1 = cdiv(T1, 16), RBW = W / 16;
  // first layer on the vector ALUs (one-hot columns are gathers), SiLU,
  // straight into LDS fragments; the radial columns of W_0 are staged in LDS
  __shared__ float w0r[T0 * 16];
  {
    const int K0 = 2 * a.S + a.nb;
    for (int q = tid; q < T0 * 16; q += NTHR) {
      const int f = q / 16, nn = q % 16;
      w0r[q] = nn < a.nb ? a.w0[(int64_t)f * K0 + 2 * a.S + nn] : 0.0f;
    }
    __syncthreads();
    constexpr int NF = cdiv(T0, 32) * NCB * 64;
    for (int idx = tid; idx < NF; idx += NTHR) {
      const int l = idx & 63, cb = (idx >> 6) % NCB, kb = idx / (64 * NCB), gl = l >> 4;
      const int64_t t = tile * TILE + 16 * cb + (l & 15);
      const bool valid = t < M;
      float rho[16];
      int zi = 0, zj = 0;
#pragma unroll
      for (int n = 0; n < 16; ++n) rho[n] = 0.0f;
      if (valid) {
        const float r = a.geo[t * GEO_STRIDE + GEO_D];
        const float ut = a.geo[t * GEO_STRIDE + GEO_U];
        const float pre = sqrtf(2.0f / a.r_cut) / r * ut;
#pragma unroll
        for (int n = 0; n < 16; ++n)
          if (n < a.nb) rho[n] = pre * __sinf((n + 1) * 3.14159265358979323846f * r / a.r_cut);
        zi = min(max(a.species[a.eidx[t]], 0), a.S - 1);
        zj = min(max(a.species[a.col[e0 + t]], 0), a.S - 1);
      }
      f32x4 v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = 32 * kb + 16 * h + 4 * gl + q;
          float sacc = 0.0f;
          if (f < T0 && valid) {
            const float* w = a.w0 + (int64_t)f * K0;
            sacc = w[zi] + w[a.S + zj];
#pragma unroll
            for (int n = 0; n < 16; ++n) sacc += w0r[f * 16 + n] * rho[n];
          }
          v[h][q] = sacc;
        }
        if (2 * kb + h < RB0) st_pre(a.pre[0], tile, RB0, 2 * kb + h, cb, l, v[h]);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[h][q] = v[h][q] * sigm(v[h][q]);
      }
      const bf16x8 hi = pack8(v[0], v[1]);
      S.act[0][idx] = __builtin_bit_cast(uint4, hi);
      S.act[0][idx + KB0 * NCB * 64] = __builtin_bit_cast(uint4, pack_rem(v[0], v[1], hi));
    }
  }
  __syncthreads();
  // hidden / output layers: SiLU; the last one x^0 = u silu(a) to HBM
  auto hidden = [&](uint2* pre, int RB, bool out_layer) {
    return [&, pre, RB, out_layer](int rb, int cb, f32x4& v) {
      if (rb >= RB) return;
      st_pre(pre, tile, RB, rb, cbA(cb), lane, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = out_layer ? u[cb] * v[q] * sigm(v[q]) : v[q] * sigm(v[q]);
      if (out_layer) {
        const int64_t t = col_t(cb);
        if (t < M) st4_stream(a.xnew + t * W + 16 * rb + 4 * g, v);
      }
    };
  };
  layer_lds<KB1, KB0, kSplit, KB0, NT == 3 ? KB1 : 0>(a.tbf[1], S.act[0], S.act[1], hidden(a.pre[1], RB1, NT == 2),
                                                     pslot, half, lane);
  __syncthreads();
  int cur = 1;
  if constexpr (NT == 3) {
    layer_lds<W / 32, KB1, kSplit, KB1>(a.tbf[2], S.act[1], S.act[0], hidden(a.pre[2], RBW, true), pslot, half, lane);
    __syncthreads();
    cur = 0;
  }
  // omega^1 = W_env^1 x^0
  layer_lds<cdiv(ENV, 32), W / 32, kSplitEnv>(
      a.envf, S.act[cur], nullptr,
      [&](int rb, int cb, f32x4& v) {
        const int64_t t = col_t(cb);
        if (rb < ENV / 16 && t < M) st_bf16x4(a.omega + t * ENV + 16 * rb + 4 * g, v);
      },
      pslot, half, lane);
}

// ---------------------------------------------------------------------------
// latent MLP of one layer (forward) + next environment embedding or energies

template <int W, int KS, int ENV, int DEPTH, bool LAST>
__global__ void __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(wpe_for<W>()))) k_lat_fwd(ChainArgs a) {
  AFM_TILE_PROLOGUE
  constexpr int RBW = W / 16, KBX = W / 32, KB0 = cdiv(W + KS, 32), NPW = W / 32;
  constexpr int NPP = cdiv(NPW, NPS);   // output-row pairs per wavefront
  static_assert(NPP == 1 || NPW % NPS == 0, "whole pairs per pair slot");
  const float r2 = 0.70710678118654752f;
  __shared__ ChainSmem<cmax(W, KS)> S;
  const bool mine = pslot < NPW;
  auto pair_of = [&](int j) { return pslot + j * NPS; };
  float ep[NCBW];
#pragma unroll
  for (int cb = 0; cb < NCBW; ++cb) ep[cb] = 0.0f;
  // x^{L-1} of the pair's rows, loaded after the last layer's MFMAs and
  // before its epilogue stores (a load behind a store the compiler cannot
  // prove disjoint waits for its own round trip: 8 serialised per pair)
  f32x4 xpf[2][NCBW];
  // epilogue of latent layer k: SiLU, or the residual update after the last
  auto epi = [&](auto K) {
    constexpr int k = decltype(K)::value;
    return [&](int rb, int cb, f32x4& v) {
      st_pre(a.pre[k], tile, RBW, rb, cbA(cb), lane, v);
      if constexpr (k < DEPTH - 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = v[q] * sigm(v[q]);
      } else {
        const int64_t t = col_t(cb);
        const bool valid = t < M;
        const f32x4 xp = xpf[rb & 1][cb];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (xp[q] + u[cb] * v[q] * sigm(v[q])) * r2;
        if constexpr (!LAST) {
          if (valid) st4_stream(a.xnew + t * W + 16 * rb + 4 * g, v);
        } else {
          const f32x4 we = ld4(a.w_eff + 16 * rb + 4 * g);
#pragma unroll
          for (int q = 0; q < 4; ++q) ep[cb] += we[q] * v[q];
        }
      }
    };
  };
  // layer 0 over [x | s]: x staged in one buffer, s in the other; the
  // output overwrites the x buffer after a barrier (so every pair of the
  // wavefront keeps its accumulators across it)
  f32x4 acc0[NPP][2][NCBW];
#pragma unroll
  for (int j = 0; j < NPP; ++j) zero_acc(acc0[j]);
  {
    // x and s loads all in flight together
    Stager<W, true> sx;
    Stager<KS, false> ss;
    sx.load(a.xprev, tile, M, tid);
    ss.load(a.s16, tile, M, tid);
    sx.store(S.act[0], tid);
    ss.store(S.act[1], tid);
  }
  __syncthreads();
  if (mine) {
#pragma unroll
    for (int j = 0; j < NPP; ++j) {
      mma_pair<KB0, KBX>(a.latf[0], pair_of(j), 0, S.act[0], acc0[j], half, lane);
      mma_pair<KB0, KB0 - KBX>(a.latf[0], pair_of(j), KBX, S.act[1], acc0[j], half, lane);
    }
  }
  __syncthreads();
  auto load_xpf = [&](int pair) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int cb = 0; cb < NCBW; ++cb) {
        const int64_t t = col_t(cb);
        xpf[r][cb] = t < M ? ld4(a.xprev + t * W + 16 * (2 * pair + r) + 4 * g) : zero4();
      }
  };
  if (mine) {
#pragma unroll
    for (int j = 0; j < NPP; ++j) {
      if constexpr (DEPTH == 1) load_xpf(pair_of(j));
      finish_pair(pair_of(j), acc0[j], (LAST && DEPTH == 1) ? nullptr : S.act[0],
                  epi(std::integral_constant<int, 0>{}), half, lane);
    }
  }
  __syncthreads();
  int cur = 0;
  static_for<1, DEPTH>([&](auto K) __attribute__((always_inline)) {
    constexpr int k = decltype(K)::value;
    if (mine) {
#pragma unroll
      for (int j = 0; j < NPP; ++j) {
        f32x4 acc[2][NCBW];
        zero_acc(acc);
        mma_pair<KBX, KBX>(a.latf[k], pair_of(j), 0, S.act[cur], acc, half, lane);
        if constexpr (k == DEPTH - 1) load_xpf(pair_of(j));
        finish_pair(pair_of(j), acc, (LAST && k == DEPTH - 1) ? nullptr : S.act[cur ^ 1], epi(K), half, lane);
      }
    }
    __syncthreads();
    cur ^= 1;
  });
  if constexpr (!LAST) {
    layer_lds<cdiv(ENV, 32), KBX, kSplitEnv>(
        a.envf, S.act[cur], nullptr,
        [&](int rb, int cb, f32x4& v) {
          const int64_t t = col_t(cb);
          if (rb < ENV / 16 && t < M) st_bf16x4(a.omega + t * ENV + 16 * rb + 4 * g, v);
        },
        pslot, half, lane);
  } else {
    // eps_e = w_eff . x^{N_L}
#pragma unroll
    for (int cb = 0; cb < NCBW; ++cb) ep[cb] = sum_groups(ep[cb]);
    wg_edge_sum(S.red, ep, tile, M, tid, [&](int64_t t, float v) { a.eps[e0 + t] = v; });
  }
}

// ---------------------------------------------------------------------------
// adjoint of one latent layer: dE/dx^L -> dE/dx^{L-1}, dE/ds^L, dE/du

template <int W, int KS, int ENV, int DEPTH, bool LAST, int kSplitBwd>
__global__ void __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(wpe_for<W>()))) k_lat_bwd(ChainArgs a) {
  AFM_TILE_PROLOGUE
  constexpr int RBW = W / 16, KBX = W / 32, NPW = W / 32;
  constexpr int NPP = cdiv(NPW, NPS);   // output-row pairs per wavefront
  static_assert(NPP == 1 || NPW % NPS == 0, "whole pairs per pair slot");
  const float r2 = 0.70710678118654752f;
  __shared__ ChainSmem<cmax(W, ENV)> S;
  const bool mine = pslot < NPW;
  auto pair_of = [&](int j) { return pslot + j * NPS; };
  float gu[NCBW];
#pragma unroll
  for (int cb = 0; cb < NCBW; ++cb) gu[cb] = 0.0f;
  // sigma_Z(i) escale gE_s of the edge in column block cb (last layer)
  auto edge_coef = [&](int cb) {
    const int64_t t = col_t(cb);
    float ce = 0.0f;
    if (t < M) {
      const int64_t i = a.eidx[t];
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
    return ce;
  };
  // head: x^L = (x^{L-1} + u silu(a_D)) / sqrt 2; v = dE/dx^L on entry.  The
  // residual share r2 v of dE/dx^{L-1} is not kept: the last layer rebuilds
  // it from w_eff at the end, the others from the stored part of gx (left
  // in place) and the environment product, formed again there
  auto head = [&](int rb, int cb, f32x4& v) {
    const f32x4 pa = ld_pre(a.pre[DEPTH - 1], tile, RBW, rb, cbA(cb), lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float gs_ = v[q] * r2;
      const float sg = sigm(pa[q]);
      gu[cb] += gs_ * pa[q] * sg;
      v[q] = gs_ * u[cb] * sg * (1.0f + pa[q] * (1.0f - sg));
    }
  };
  if constexpr (LAST) {
    // dE/dx^{N_L} = sigma_Z(i) escale gE_s w_eff
    if (mine) {
      float ce[NCBW];
#pragma unroll
      for (int cb = 0; cb < NCBW; ++cb) ce[cb] = edge_coef(cb);
#pragma unroll
      for (int j = 0; j < NPP; ++j) {
        f32x4 acc[2][NCBW];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const f32x4 we = ld4(a.w_eff + 16 * (2 * pair_of(j) + r) + 4 * g);
#pragma unroll
          for (int cb = 0; cb < NCBW; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[r][cb][q] = ce[cb] * we[q];
        }
        finish_pair(pair_of(j), acc, S.act[0], head, half, lane);
      }
    }
  } else {
    // dE/dx^L = (stored) + W_env^{L+1 T} dE/domega^{L+1}
    stage_rows_bf16<ENV>(S.act[1], a.gomega, tile, M, tid);
    __syncthreads();
    if (mine) {
#pragma unroll
      for (int j = 0; j < NPP; ++j) {
        f32x4 acc[2][NCBW];
        zero_acc(acc);
        mma_pair<cdiv(ENV, 32), cdiv(ENV, 32), kSplitEnv>(a.envb, pair_of(j), 0, S.act[1], acc, half, lane);
        finish_pair(
            pair_of(j), acc, S.act[0],
            [&](int rb, int cb, f32x4& v) {
              const int64_t t = col_t(cb);
              if (t < M) v += ld4(a.gx + t * W + 16 * rb + 4 * g);
              head(rb, cb, v);
            },
            half, lane);
      }
    }
  }
#pragma unroll
  for (int cb = 0; cb < NCBW; ++cb) gu[cb] = sum_groups(gu[cb]);
  // (the barrier inside also publishes the head's fragments)
  wg_edge_sum(S.red, gu, tile, M, tid, [&](int64_t t, float v) { a.gy[t * GEO_STRIDE + 9] += v; });
  // inner layers: ga_{k-1} = (W_k^T ga_k) * silu'(a_{k-1})
  int cur = 0;
  static_for<1, DEPTH>([&](auto KK) __attribute__((always_inline)) {
    constexpr int k = DEPTH - decltype(KK)::value;
    if (mine) {
#pragma unroll
      for (int j = 0; j < NPP; ++j) {
        f32x4 acc[2][NCBW];
        zero_acc(acc);
        mma_pair<KBX, KBX, kSplitBwd>(a.latb[k], pair_of(j), 0, S.act[cur], acc, half, lane);
        finish_pair(
            pair_of(j), acc, S.act[cur ^ 1],
            [&](int rb, int cb, f32x4& v) {
              const f32x4 pa = ld_pre(a.pre[k - 1], tile, RBW, rb, cbA(cb), lane);
#pragma unroll
              for (int q = 0; q < 4; ++q) v[q] *= dsilu_of(pa[q]);
            },
            half, lane);
      }
    }
    __syncthreads();
    cur ^= 1;
  });
  // dE/d[x | s] = W_1^T ga_1: x rows added to the residual share, s rows
  // stored.  Not in the last layer, the x rows' accumulators start from
  // r2 W_env^T dE/domega (dE/domega staged again into the free buffer), and
  // the epilogue adds r2 x the stored part of gx.
  if constexpr (!LAST) {
    restage_rows_bf16<ENV>(S.act[cur ^ 1], a.gomega, tile, M, tid);
    __syncthreads();
  }
  // a fresh copy of the tile index, so that the compiler forms the edge
  // indices and addresses anew here instead of keeping the head's 64-bit
  // ones live (spilled) across the whole chain
  int64_t tile_o = tile;
  asm volatile("" : "+s"(tile_o));
  auto out_epi = [&](int rb, int cb, f32x4& v) {
    const int64_t t = tile_o * TILE + 16 * cbA(cb) + (lane & 15);
    if (t >= M) return;
    if (rb < RBW) {
      float* p = a.gx + t * W + 16 * rb + 4 * g;
      f32x4 res;
      if constexpr (LAST) {
        const float ce = edge_coef(cb);
        const f32x4 we = ld4(a.w_eff + 16 * rb + 4 * g);
#pragma unroll
        for (int q = 0; q < 4; ++q) res[q] = (ce * we[q]) * r2;
      } else {
        res = ld4(p) * r2;
      }
      st4(p, res + v);
    } else if (16 * (rb - RBW) < KS) {
      st_bf16x4_plain(a.gs + t * KS + 16 * (rb - RBW) + 4 * g, v);
    }
  };
  constexpr int NPO = cdiv(W + KS, 32);
  static_for<0, cdiv(NPO, NPS)>([&](auto P) __attribute__((always_inline)) {
    const int p = decltype(P)::value * NPS + pslot;
    if (p < NPO) {
      f32x4 acc[2][NCBW];
      zero_acc(acc);
      if constexpr (!LAST) {
        if (p < NPW) {
          mma_pair<cdiv(ENV, 32), cdiv(ENV, 32), kSplitEnv>(a.envb, p, 0, S.act[cur ^ 1], acc, half, lane);
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < NCBW; ++c) acc[r][c] *= r2;
        }
      }
      mma_pair<KBX, KBX, kSplitBwd>(a.latb[0], p, 0, S.act[cur], acc, half, lane);
      finish_pair(p, acc, nullptr, out_epi, half, lane);
    }
  });
}

#ifdef AFM_TILE_FUSED
// ---------------------------------------------------------------------------
// The last latent layer's forward and adjoint in one kernel.  Its adjoint
// seed dE/dx^{N_L} = sigma_Z(i) escale gE_s w_eff is known per edge before
// the layer runs, so the adjoint head is applied in the forward's last
// epilogue on the same registers (to the bf16-rounded pre-activation, as
// the separate adjoint reads it), and the inner layers' pre-activations
// stay in LDS instead of going to HBM and back: the results are bitwise
// those of k_lat_fwd + k_lat_bwd.  Needs 130 KB of LDS at w = 256, so one
// workgroup per CU.
template <int W, int KS, int DEPTH, int kSplitBwd>
__global__ void __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(2))) k_lat_fb(ChainArgs a) {
  AFM_TILE_PROLOGUE
  static_assert(W <= 32 * NPS, "one output-row pair per wavefront");
  constexpr int RBW = W / 16, KBX = W / 32, KB0 = cdiv(W + KS, 32), NPW = W / 32;
  const float r2 = 0.70710678118654752f;
  __shared__ ChainSmem<cmax(W, KS)> S;
  __shared__ uint2 PRE[DEPTH > 1 ? DEPTH - 1 : 1][RBW * NCB * 64];
  const bool mine = pslot < NPW;
  const int pair = pslot;
  // sigma_Z(i) escale gE_s of the edge in column block cb
  float ce[NCBW], ep[NCBW], gu[NCBW];
#pragma unroll
  for (int cb = 0; cb < NCBW; ++cb) {
    ep[cb] = 0.0f;
    gu[cb] = 0.0f;
    const int64_t t = col_t(cb);
    ce[cb] = 0.0f;
    if (t < M) {
      const int64_t i = a.eidx[t];
      ce[cb] = (float)(a.sp_scale[min(max(a.species[i], 0), a.S - 1)] * a.escale);
      if (a.ges) {
        int64_t lo = 0, hi = a.B;
        while (hi - lo > 1) {
          int64_t mid = (lo + hi) >> 1;
          if (a.seg[mid] <= i) lo = mid; else hi = mid;
        }
        ce[cb] *= (float)a.ges[lo];
      }
    }
  }
  auto pre_idx = [&](int rb, int cb) { return (rb * NCB + cbA(cb)) * 64 + lane; };
  f32x4 xpf[2][NCBW];
  auto epi = [&](auto K) {
    constexpr int k = decltype(K)::value;
    return [&](int rb, int cb, f32x4& v) {
      if constexpr (k < DEPTH - 1) {
        bf16x4 h;
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = (__bf16)v[q];
        PRE[k][pre_idx(rb, cb)] = __builtin_bit_cast(uint2, h);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = v[q] * sigm(v[q]);
      } else {
        const f32x4 xp = xpf[rb & 1][cb];
        const f32x4 we = ld4(a.w_eff + 16 * rb + 4 * g);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // energy: x^{N_L} and its edge-energy product
          const float xl = (xp[q] + u[cb] * v[q] * sigm(v[q])) * r2;
          ep[cb] += we[q] * xl;
          // adjoint head on the bf16 pre-activation
          const float pa = (float)(__bf16)v[q];
          const float gs_ = (ce[cb] * we[q]) * r2;
          const float sg = sigm(pa);
          gu[cb] += gs_ * pa * sg;
          v[q] = gs_ * u[cb] * sg * (1.0f + pa * (1.0f - sg));
        }
      }
    };
  };
  auto load_xpf = [&]() {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int cb = 0; cb < NCBW; ++cb) {
        const int64_t t = col_t(cb);
        xpf[r][cb] = t < M ? ld4(a.xprev + t * W + 16 * (2 * pair + r) + 4 * g) : zero4();
      }
  };
  // forward: layer 0 over [x | s]
  f32x4 acc0[2][NCBW];
  zero_acc(acc0);
  {
    Stager<W, true> sx;
    Stager<KS, false> ss;
    sx.load(a.xprev, tile, M, tid);
    ss.load(a.s16, tile, M, tid);
    sx.store(S.act[0], tid);
    ss.store(S.act[1], tid);
  }
  __syncthreads();
  if (mine) {
    mma_pair<KB0, KBX>(a.latf[0], pair, 0, S.act[0], acc0, half, lane);
    mma_pair<KB0, KB0 - KBX>(a.latf[0], pair, KBX, S.act[1], acc0, half, lane);
  }
  __syncthreads();
  if (mine) {
    if constexpr (DEPTH == 1) load_xpf();
    finish_pair(pair, acc0, S.act[0], epi(std::integral_constant<int, 0>{}), half, lane);
  }
  __syncthreads();
  int cur = 0;
  static_for<1, DEPTH>([&](auto K) __attribute__((always_inline)) {
    constexpr int k = decltype(K)::value;
    if (mine) {
      f32x4 acc[2][NCBW];
      zero_acc(acc);
      mma_pair<KBX, KBX>(a.latf[k], pair, 0, S.act[cur], acc, half, lane);
      if constexpr (k == DEPTH - 1) load_xpf();
      finish_pair(pair, acc, S.act[cur ^ 1], epi(K), half, lane);
    }
    __syncthreads();
    cur ^= 1;
  });
  // edge energies and dE/du of the head (the barriers inside also publish
  // the head's fragments)
#pragma unroll
  for (int cb = 0; cb < NCBW; ++cb) ep[cb] = sum_groups(ep[cb]);
  wg_edge_sum(S.red, ep, tile, M, tid, [&](int64_t t, float v) { a.eps[e0 + t] = v; });
#pragma unroll
  for (int cb = 0; cb < NCBW; ++cb) gu[cb] = sum_groups(gu[cb]);
  wg_edge_sum(S.red, gu, tile, M, tid, [&](int64_t t, float v) { a.gy[t * GEO_STRIDE + 9] += v; });
  // adjoint: inner layers ga_{k-1} = (W_k^T ga_k) * silu'(a_{k-1})
  static_for<1, DEPTH>([&](auto KK) __attribute__((always_inline)) {
    constexpr int k = DEPTH - decltype(KK)::value;
    if (mine) {
      f32x4 acc[2][NCBW];
      zero_acc(acc);
      mma_pair<KBX, KBX, kSplitBwd>(a.latb[k], pair, 0, S.act[cur], acc, half, lane);
      finish_pair(
          pair, acc, S.act[cur ^ 1],
          [&](int rb, int cb, f32x4& v) {
            const bf16x4 h = __builtin_bit_cast(bf16x4, PRE[k - 1][pre_idx(rb, cb)]);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] *= dsilu_of((float)h[q]);
          },
          half, lane);
    }
    __syncthreads();
    cur ^= 1;
  });
  // dE/d[x | s] = W_1^T ga_1: x rows plus the residual share, s rows stored
  int64_t tile_o = tile;
  asm volatile("" : "+s"(tile_o));
  auto out_epi = [&](int rb, int cb, f32x4& v) {
    const int64_t t = tile_o * TILE + 16 * cbA(cb) + (lane & 15);
    if (t >= M) return;
    if (rb < RBW) {
      const f32x4 we = ld4(a.w_eff + 16 * rb + 4 * g);
      f32x4 res;
#pragma unroll
      for (int q = 0; q < 4; ++q) res[q] = (ce[cb] * we[q]) * r2;
      st4(a.gx + t * W + 16 * rb + 4 * g, res + v);
    } else if (16 * (rb - RBW) < KS) {
      st_bf16x4_plain(a.gs + t * KS + 16 * (rb - RBW) + 4 * g, v);
    }
  };
  constexpr int NPO = cdiv(W + KS, 32);
  static_for<0, cdiv(NPO, NPS)>([&](auto P) __attribute__((always_inline)) {
    const int p = decltype(P)::value * NPS + pslot;
    if (p < NPO) {
      f32x4 acc[2][NCBW];
      zero_acc(acc);
      mma_pair<KBX, KBX, kSplitBwd>(a.latb[0], p, 0, S.act[cur], acc, half, lane);
      finish_pair(p, acc, nullptr, out_epi, half, lane);
    }
  });
}
#endif

// ---------------------------------------------------------------------------
// adjoint of the two-body MLP: dE/dx^0 (+ W_env^1T dE/domega^1) -> dE/drho, dE/du

template <int T0, int T1, int T2, int W, int ENV, int kSplitBwd>
__global__ void __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(wpe_for<W>()))) k_tb_bwd(ChainArgs a) {
  AFM_TILE_PROLOGUE
  constexpr int NT = T2 ? 3 : 2;
  constexpr int RBW = W / 16, RB0 = cdiv(T0, 16), RB1 = cdiv(T1, 16), NPW = W / 32;
  constexpr int NPP = cdiv(NPW, NPS);   // output-row pairs per wavefront
  static_assert(NPP == 1 || NPW % NPS == 0, "whole pairs per pair slot");
  __shared__ ChainSmem<cmax(cmax(ENV, W), T1)> S;
  const bool mine = pslot < NPW;
  float gu[NCBW];
#pragma unroll
  for (int cb = 0; cb < NCBW; ++cb) gu[cb] = 0.0f;
  // head: x^0 = u silu(a_last); dE/dx^0 = stored + W_env^1T dE/domega^1
  stage_rows_bf16<ENV>(S.act[1], a.gomega, tile, M, tid);
  __syncthreads();
  if (mine) {
#pragma unroll
  for (int j = 0; j < NPP; ++j) {
    const int pair = pslot + j * NPS;
    f32x4 acc[2][NCBW];
    zero_acc(acc);
    mma_pair<cdiv(ENV, 32), cdiv(ENV, 32), kSplitEnv>(a.envb, pair, 0, S.act[1], acc, half, lane);
    finish_pair(
        pair, acc, S.act[0],
        [&](int rb, int cb, f32x4& v) {
          const int64_t t = col_t(cb);
          const f32x4 gx = t < M ? ld4(a.gx + t * W + 16 * rb + 4 * g) : zero4();
          const f32x4 pa = ld_pre(a.pre[NT - 1], tile, RBW, rb, cbA(cb), lane);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float gv = v[q] + gx[q];
            const float sg = sigm(pa[q]);
            gu[cb] += gv * pa[q] * sg;
            v[q] = gv * u[cb] * sg * (1.0f + pa[q] * (1.0f - sg));
          }
        },
        half, lane);
  }
  }
#pragma unroll
  for (int cb = 0; cb < NCBW; ++cb) gu[cb] = sum_groups(gu[cb]);
  wg_edge_sum(S.red, gu, tile, M, tid, [&](int64_t t, float v) { a.gy[t * GEO_STRIDE + 9] += v; });
  int cur = 0;
  if constexpr (NT == 3) {
    layer_lds<cdiv(T1, 32), W / 32, kSplitBwd>(
        a.tbb[2], S.act[0], S.act[1],
        [&](int rb, int cb, f32x4& v) {
          if (rb >= RB1) return;
          const f32x4 pa = ld_pre(a.pre[1], tile, RB1, rb, cbA(cb), lane);
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] *= dsilu_of(pa[q]);
        },
        pslot, half, lane);
    __syncthreads();
    cur = 1;
  }
  // ga_0 = (W_1^T ga_1) * silu'(a_0), then dE/drho_n = sum_f W_0[f][2S + n] ga_0[f]
  constexpr int NP0 = cdiv(T0, 32);
  static_assert(NP0 <= NPS, "one pair per pair slot");
  f32x4 acc[2][NCBW];
  zero_acc(acc);
  if (pslot < NP0) {
    mma_pair<cdiv(T1, 32), cdiv(T1, 32), kSplitBwd>(a.tbb[1], pslot, 0, S.act[cur], acc, half, lane);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int rb = 2 * pslot + r;
#pragma unroll
      for (int cb = 0; cb < NCBW; ++cb) {
        if (rb < RB0) {
          const f32x4 pa = ld_pre(a.pre[0], tile, RB0, rb, cbA(cb), lane);
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[r][cb][q] *= dsilu_of(pa[q]);
        } else {
          acc[r][cb] = zero4();
        }
      }
    }
  }
  const int K0 = 2 * a.S + a.nb;
  // radial columns of W_0
  __shared__ float w0r[T0 * 16];
  for (int q = tid; q < T0 * 16; q += NTHR) {
    const int f = q / 16, nn = q % 16;
    w0r[q] = nn < a.nb ? a.w0[(int64_t)f * K0 + 2 * a.S + nn] : 0.0f;
  }
  __syncthreads();
  // this wavefront's share of sum_f W_0[f][2S + n] ga_0[f] for column block cb
  auto rho_part = [&](int n, int cb) {
    float p = 0.0f;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = 16 * (2 * pslot + r) + 4 * g + q;
        if (f < T0) p += w0r[f * 16 + n] * acc[r][cb][q];
      }
    return sum_groups(p);
  };
  constexpr bool kOnePass = sizeof(S.act) >= sizeof(float) * NP0 * 16 * TILE;
  if constexpr (kOnePass) {
    // all radial channels at once: the activation buffers are free after
    // the barrier above and hold the [pair slot][n][edge] partials, summed
    // over the pair slots in slot order
    float* red = reinterpret_cast<float*>(&S.act[0][0]);
    if (pslot < NP0) {
      for (int n = 0; n < a.nb; ++n)
#pragma unroll
        for (int cb = 0; cb < NCBW; ++cb) {
          const float v = rho_part(n, cb);
          if (g == 0) red[(pslot * 16 + n) * TILE + 16 * cbA(cb) + lane] = v;
        }
    }
    __syncthreads();
    for (int idx = tid; idx < a.nb * TILE; idx += NTHR) {
      const int e = idx / a.nb, n = idx % a.nb;
      float v = 0.0f;
#pragma unroll
      for (int w = 0; w < NP0; ++w) v += red[(w * 16 + n) * TILE + e];
      const int64_t t = tile * TILE + e;
      if (t < M) a.grho[t * 16 + n] = v;
    }
  } else {
    for (int n = 0; n < a.nb; ++n) {
      float part[NCBW];
#pragma unroll
      for (int cb = 0; cb < NCBW; ++cb) part[cb] = pslot < NP0 ? rho_part(n, cb) : 0.0f;
      wg_edge_sum(S.red, part, tile, M, tid, [&](int64_t t, float v) { a.grho[t * 16 + n] = v; });
    }
  }
}

// ---------------------------------------------------------------------------
// launchers for this tile shape (arguments prepared by the caller)

static dim3 chain_grid(const WsLayout& L) { return dim3(grid_for(L.cex, TILE)); }

static int launch_tb_fwd(const ModelDims& d, const ChainArgs& a, const WsLayout& L, hipStream_t st) {
#define X(w, c, l, dp, a0, a1, a2, n0)                                                             \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                  \
    hipLaunchKernelGGL((k_tb_fwd<a0, a1, a2, w, (l + 1) * c>), chain_grid(L), dim3(NTHR), 0, st, a); \
    AFM_LAUNCH_CHECK();                                                                            \
    return AFM_OK;                                                                                 \
  }
  AFM_SHAPES(X)
#ifdef AFM_TILE_WIDE
  AFM_SHAPES_WIDE(X)
#endif
#undef X
  return AFM_E_UNSUPPORTED;
}

static int launch_tb_bwd(const ModelDims& d, bool fast, const ChainArgs& a, const WsLayout& L, hipStream_t st) {
#define X(w, c, l, dp, a0, a1, a2, n0)                                                             \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                  \
    if (fast)                                                                                      \
      hipLaunchKernelGGL((k_tb_bwd<a0, a1, a2, w, (l + 1) * c, 1>), chain_grid(L), dim3(NTHR), 0, st, a); \
    else                                                                                           \
      hipLaunchKernelGGL((k_tb_bwd<a0, a1, a2, w, (l + 1) * c, kSplit>), chain_grid(L), dim3(NTHR), 0, st, a); \
    AFM_LAUNCH_CHECK();                                                                            \
    return AFM_OK;                                                                                 \
  }
  AFM_SHAPES(X)
#ifdef AFM_TILE_WIDE
  AFM_SHAPES_WIDE(X)
#endif
#undef X
  return AFM_E_UNSUPPORTED;
}

static int launch_lat_fwd(const ModelDims& d, bool last, const ChainArgs& a, const WsLayout& L, hipStream_t st) {
#define X(w, c, l, dp, a0, a1, a2, n0)                                                                  \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                       \
    if (last)                                                                                           \
      hipLaunchKernelGGL((k_lat_fwd<w, n0 * c, (l + 1) * c, dp, true>), chain_grid(L), dim3(NTHR), 0, st, a);  \
    else                                                                                                \
      hipLaunchKernelGGL((k_lat_fwd<w, n0 * c, (l + 1) * c, dp, false>), chain_grid(L), dim3(NTHR), 0, st, a); \
    AFM_LAUNCH_CHECK();                                                                                 \
    return AFM_OK;                                                                                      \
  }
  AFM_SHAPES(X)
#ifdef AFM_TILE_WIDE
  AFM_SHAPES_WIDE(X)
#endif
#undef X
  return AFM_E_UNSUPPORTED;
}

static int launch_lat_bwd(const ModelDims& d, bool last, bool fast, const ChainArgs& a, const WsLayout& L,
                          hipStream_t st) {
#define X(w, c, l, dp, a0, a1, a2, n0)                                                                  \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                       \
    if (last && fast)                                                                                   \
      hipLaunchKernelGGL((k_lat_bwd<w, n0 * c, (l + 1) * c, dp, true, 1>), chain_grid(L), dim3(NTHR), 0, st, a); \
    else if (last)                                                                                      \
      hipLaunchKernelGGL((k_lat_bwd<w, n0 * c, (l + 1) * c, dp, true, kSplit>), chain_grid(L), dim3(NTHR), 0, st, \
                         a);                                                                            \
    else if (fast)                                                                                      \
      hipLaunchKernelGGL((k_lat_bwd<w, n0 * c, (l + 1) * c, dp, false, 1>), chain_grid(L), dim3(NTHR), 0, st, a); \
    else                                                                                                \
      hipLaunchKernelGGL((k_lat_bwd<w, n0 * c, (l + 1) * c, dp, false, kSplit>), chain_grid(L), dim3(NTHR), 0, st, \
                         a);                                                                            \
    AFM_LAUNCH_CHECK();                                                                                 \
    return AFM_OK;                                                                                      \
  }
  AFM_SHAPES(X)
#ifdef AFM_TILE_WIDE
  AFM_SHAPES_WIDE(X)
#endif
#undef X
  return AFM_E_UNSUPPORTED;
}

#ifdef AFM_TILE_FUSED
static int launch_lat_fb(const ModelDims& d, bool fast, const ChainArgs& a, const WsLayout& L, hipStream_t st) {
#define X(w, c, l, dp, a0, a1, a2, n0)                                                                  \
  if (shape_is(d, w, c, l, dp, a0, a1, a2, n0)) {                                                       \
    if (fast)                                                                                           \
      hipLaunchKernelGGL((k_lat_fb<w, n0 * c, dp, 1>), chain_grid(L), dim3(NTHR), 0, st, a);            \
    else                                                                                                \
      hipLaunchKernelGGL((k_lat_fb<w, n0 * c, dp, kSplit>), chain_grid(L), dim3(NTHR), 0, st, a);       \
    AFM_LAUNCH_CHECK();                                                                                 \
    return AFM_OK;                                                                                      \
  }
  AFM_SHAPES(X)
#undef X
  return AFM_E_UNSUPPORTED;
}
#endif

#undef AFM_TILE_PROLOGUE
