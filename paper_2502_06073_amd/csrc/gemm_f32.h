// FP32 GEMMs on the vector ALUs (plain-FP32 path and second-order path).
//
// k_sgemm:  C[m][n] = sum_k A(m, k) * B(k, n) over the rows of the current
// chunk, A read through a loader functor (concatenations, SiLU on load), B a
// row-major weight matrix used as W^T ([N][K], "NT") or W ([K][N], "NN"),
// and a fused epilogue functor.  With stack > 0 the rows are "stacked":
// [0, stack) and [stack, 2 stack) are two row sets (primal and tangent)
// sharing the weights; row m is live if m % stack < rows of the chunk.
// 64 x 64 tiles, K steps of 16 staged in LDS, 4 x 4 outputs per thread.
//
// k_wgrad:  P[slice][n][k] = sum_{m in slice} A(m, n) * B(m, k): weight
// gradients reduced over edges; slices are summed afterwards in a fixed
// order (deterministic, no atomics).
//
// The _mfma variants (second-order path) stage the same LDS tiles and
// multiply them on the matrix cores in FP32 (v_mfma_f32_16x16x4f32, FP32
// products and accumulation): each of the 4 wavefronts owns a 32 x 32
// quarter of the tile as 2 x 2 blocks of 16 x 16.  The _bf16 variants (the
// second-order path of BF16 models) round both operands to bf16 when they
// are staged and multiply on v_mfma_f32_16x16x32_bf16 (FP32 accumulation):
// a stage covers 32 of the reduction index, held as rows of 8 consecutive
// values per lane group.
#pragma once
#include <hip/hip_runtime.h>

#include "edge_layout.h"

namespace afm {

__device__ __forceinline__ bool row_live(int m, int M, int stack) {
  return stack ? (m % stack) < M : m < M;
}

template <bool NT, class AL, class EP>
__global__ void __launch_bounds__(256) k_sgemm(RowRange rr, int K, int N, const float* __restrict__ W, int ldw,
                                               AL al, EP ep, int stack) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int rows = stack ? 2 * stack : M;
  const int m0 = blockIdx.x * 64;
  if (m0 >= rows) return;
  // stack is a multiple of 64, so a 64-row block lies in one row set
  if (stack && (m0 % stack) >= M) return;
  const int n0 = blockIdx.y * 64;
  __shared__ float As[16][68];
  __shared__ float Bs[16][68];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx >> 4, kk = idx & 15;
      const int m = m0 + r, k = k0 + kk;
      As[kk][r] = (m < rows && row_live(m, M, stack) && k < K) ? al(m, k) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      int kk, c;
      if (NT) { c = idx >> 4; kk = idx & 15; } else { kk = idx >> 6; c = idx & 63; }
      const int k = k0 + kk, n = n0 + c;
      float v = 0.0f;
      if (k < K && n < N) v = NT ? W[(int64_t)n * ldw + k] : W[(int64_t)k * ldw + n];
      Bs[kk][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= rows || !row_live(m, M, stack)) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n < N) ep(m, n, acc[i][j]);
    }
  }
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// A (16 x 4) and B (4 x 16) operands: lane l holds row / column l % 16 at
// k = l / 16; the 16 x 16 result: lane l holds column l % 16, rows
// 4 (l / 16) .. 4 (l / 16) + 3.
__device__ __forceinline__ f32x4_t mfma_f32(float a, float b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <bool NT, class AL, class EP>
__global__ void __launch_bounds__(256) k_sgemm_mfma(RowRange rr, int K, int N, const float* __restrict__ W, int ldw,
                                                    AL al, EP ep, int stack) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int rows = stack ? 2 * stack : M;
  const int m0 = blockIdx.x * 64;
  if (m0 >= rows) return;
  if (stack && (m0 % stack) >= M) return;
  const int n0 = blockIdx.y * 64;
  constexpr int KS = 32;  // k per stage
  __shared__ float As[KS][68];
  __shared__ float Bs[KS][68];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int lr = lane & 15, lk = lane >> 4;
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  // the next stage is fetched into registers while the current one is
  // multiplied
  float ra[KS / 4], rb[KS / 4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < KS / 4; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / KS, kk = idx % KS;
      const int m = m0 + r, k = k0 + kk;
      ra[q] = (m < rows && row_live(m, M, stack) && k < K) ? al(m, k) : 0.0f;
      int kb, c;
      if (NT) { c = idx / KS; kb = idx % KS; } else { kb = idx >> 6; c = idx & 63; }
      const int k2 = k0 + kb, n = n0 + c;
      float v = 0.0f;
      if (k2 < K && n < N) v = NT ? W[(int64_t)n * ldw + k2] : W[(int64_t)k2 * ldw + n];
      rb[q] = v;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += KS) {
#pragma unroll
    for (int q = 0; q < KS / 4; ++q) {
      const int idx = tid + 256 * q;
      As[idx % KS][idx / KS] = ra[q];
      if (NT) Bs[idx % KS][idx / KS] = rb[q]; else Bs[idx >> 6][idx & 63] = rb[q];
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
      if (m >= rows || !row_live(m, M, stack)) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + 32 * wc + 16 * j + lr;
        if (n < N) ep(m, n, acc[i][j][q]);
      }
    }
}

template <bool NT, bool MF = false, class AL, class EP>
inline void sgemm(hipStream_t st, RowRange rr, int64_t max_rows, int K, int N, const float* W, int ldw, AL al,
                  EP ep, int stack = 0) {
  const int64_t rows = stack ? 2 * (int64_t)stack : max_rows;
  dim3 grid((unsigned)((rows + 63) / 64 > 0 ? (rows + 63) / 64 : 1), (unsigned)((N + 63) / 64));
  if constexpr (MF)
    hipLaunchKernelGGL((k_sgemm_mfma<NT, AL, EP>), grid, dim3(256), 0, st, rr, K, N, W, ldw, al, ep, stack);
  else
    hipLaunchKernelGGL((k_sgemm<NT, AL, EP>), grid, dim3(256), 0, st, rr, K, N, W, ldw, al, ep, stack);
}

template <class ALA, class ALB>
__global__ void __launch_bounds__(256) k_wgrad(RowRange rr, int stack, int N, int K, int rows_per_slice,
                                               ALA A, ALB Bl, float* __restrict__ partial) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int rows = stack ? 2 * stack : M;
  const int n0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
  const int slice = blockIdx.z;
  const int r0 = slice * rows_per_slice;
  const int r1 = min(rows, r0 + rows_per_slice);
  __shared__ float As[16][68];
  __shared__ float Bs[16][68];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  float acc[4][4] = {};
  for (int m0 = r0; m0 < r1; m0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int mm = idx >> 6, c = idx & 63;
      const int m = m0 + mm;
      const bool live = m < r1 && row_live(m, M, stack);
      As[mm][c] = (live && n0 + c < N) ? A(m, n0 + c) : 0.0f;
      Bs[mm][c] = (live && k0 + c < K) ? Bl(m, k0 + c) : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[mm][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[mm][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  float* P = partial + (int64_t)slice * N * K;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int n = n0 + ty * 4 + i;
    if (n >= N) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + tx * 4 + j;
      if (k < K) P[(int64_t)n * K + k] = acc[i][j];
    }
  }
}

template <class ALA, class ALB>
__global__ void __launch_bounds__(256) k_wgrad_mfma(RowRange rr, int stack, int N, int K, int rows_per_slice,
                                                    ALA A, ALB Bl, float* __restrict__ partial) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int rows = stack ? 2 * stack : M;
  const int n0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
  const int slice = blockIdx.z;
  const int r0 = slice * rows_per_slice;
  const int r1 = min(rows, r0 + rows_per_slice);
  constexpr int MS = 32;  // rows (the reduction index) per stage
  __shared__ float As[MS][68];
  __shared__ float Bs[MS][68];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int lr = lane & 15, lk = lane >> 4;
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  float ra[MS / 4], rb[MS / 4];
  auto fetch = [&](int m0) {
#pragma unroll
    for (int q = 0; q < MS / 4; ++q) {
      const int idx = tid + 256 * q;
      const int mm = idx >> 6, c = idx & 63;
      const int m = m0 + mm;
      const bool live = m < r1 && row_live(m, M, stack);
      ra[q] = (live && n0 + c < N) ? A(m, n0 + c) : 0.0f;
      rb[q] = (live && k0 + c < K) ? Bl(m, k0 + c) : 0.0f;
    }
  };
  if (r0 < r1) fetch(r0);
  for (int m0 = r0; m0 < r1; m0 += MS) {
#pragma unroll
    for (int q = 0; q < MS / 4; ++q) {
      const int idx = tid + 256 * q;
      As[idx >> 6][idx & 63] = ra[q];
      Bs[idx >> 6][idx & 63] = rb[q];
    }
    __syncthreads();
    if (m0 + MS < r1) fetch(m0 + MS);
#pragma unroll
    for (int s4 = 0; s4 < MS / 4; ++s4) {
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
  float* P = partial + (int64_t)slice * N * K;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = n0 + 32 * wr + 16 * i + 4 * lk + q;
      if (n >= N) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int k = k0 + 32 * wc + 16 * j + lr;
        if (k < K) P[(int64_t)n * K + k] = acc[i][j][q];
      }
    }
}

// ---------------------------------------------------------------------------
// BF16 MFMA variants

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4_t mfma_bf16(bf16x8_t a, bf16x8_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// LDS tile of 64 rows x 32 reduction values in bf16, rows padded to 40
// values (80 bytes) so a lane's 8 values are one aligned 16-byte read.
constexpr int kBfRow = 40;

// 8 bf16 values [8 g, 8 g + 8) of row r
__device__ __forceinline__ bf16x8_t lds_row8(const __bf16* T, int r, int g) {
  return *reinterpret_cast<const bf16x8_t*>(T + r * kBfRow + 8 * g);
}

// BN output columns per workgroup (64 or 128): with 128 a wavefront owns
// 32 x 64 of the tile, so every A element (whose loader may apply SiLU or
// gather a concatenation) is loaded once for up to 128 outputs, and each
// staged k-step feeds twice the MFMAs; the sequence of products into every
// output is the same for both widths.  (The weight-gradient kernel below
// keeps 64 x 64 tiles and 32-row stages: 128-wide tiles, which halve its
// workgroups, and 64-row stages, which double its registers, both measured
// 7-11 % slower on the training step; with 16-byte LDS staging, 64-row
// stages (78 registers, 5 waves per SIMD instead of 8) measured the same.  64-value stages here, which halve
// the barriers per product, need 140 registers instead of 74 and measured
// 8 % slower.)
template <bool NT, int BN, class AL, class EP>
__global__ void __launch_bounds__(256) k_sgemm_bf16(RowRange rr, int K, int N, const float* __restrict__ W, int ldw,
                                                    AL al, EP ep, int stack) {
  static_assert(BN == 64 || BN == 128, "BN");
  constexpr int NJ = BN / 32;   // 16-column blocks per wavefront
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int rows = stack ? 2 * stack : M;
  const int m0 = blockIdx.x * 64;
  if (m0 >= rows) return;
  if (stack && (m0 % stack) >= M) return;
  const int n0 = blockIdx.y * BN;
  constexpr int KS = 32;
  __shared__ __attribute__((aligned(16))) __bf16 As[64 * kBfRow];   // [m][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN * kBfRow];   // [n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int lr = lane & 15, lg = lane >> 4;
  f32x4_t acc[2][NJ];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  // next stage fetched into registers while the current one is multiplied.
  // Every thread stages groups of 8 consecutive reduction values and writes
  // each group to LDS as one 16-byte store.  A: row tid / 4, values
  // 8 (tid % 4) ..; W (NT, [n][k]): rows tid / 4 + 64 h, likewise; W
  // ([k][n]): column tid % BN, values 8 (tid / BN + (256 / BN) h) ..
  constexpr int HB = BN / 64;   // W groups per thread per stage
  float ra[8], rb[HB][8];
  const int ar = tid >> 2, akq = (tid & 3) * 8;
  auto fetch = [&](int k0) {
    {
      const int m = m0 + ar, kb = k0 + akq;
      const bool live = m < rows && row_live(m, M, stack);
      if (live && kb + 8 <= K) {   // whole group in range: the loader's unguarded 8-value load
        al.load8(m, kb, ra);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) ra[q] = (live && kb + q < K) ? al(m, kb + q) : 0.0f;
      }
    }
#pragma unroll
    for (int h = 0; h < HB; ++h) {
      int c, kq;
      if (NT) { c = ar + 64 * h; kq = akq; } else { c = tid % BN; kq = 8 * (tid / BN + (256 / BN) * h); }
      const int n = n0 + c, kb = k0 + kq;
      if (NT && n < N && kb + 8 <= K) {
#pragma unroll
        for (int q = 0; q < 8; ++q) rb[h][q] = W[(int64_t)n * ldw + kb + q];
        continue;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float v = 0.0f;
        if (kb + q < K && n < N) v = NT ? W[(int64_t)n * ldw + kb + q] : W[(int64_t)(kb + q) * ldw + n];
        rb[h][q] = v;
      }
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += KS) {
    {
      bf16x8_t v;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (__bf16)ra[q];
      *reinterpret_cast<bf16x8_t*>(As + ar * kBfRow + akq) = v;
    }
#pragma unroll
    for (int h = 0; h < HB; ++h) {
      int c, kq;
      if (NT) { c = ar + 64 * h; kq = akq; } else { c = tid % BN; kq = 8 * (tid / BN + (256 / BN) * h); }
      bf16x8_t v;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (__bf16)rb[h][q];
      *reinterpret_cast<bf16x8_t*>(Bs + c * kBfRow + kq) = v;
    }
    __syncthreads();
    if (k0 + KS < K) fetch(k0 + KS);
    bf16x8_t a[2], b[NJ];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = lds_row8(As, 32 * wr + 16 * i + lr, lg);
#pragma unroll
    for (int j = 0; j < NJ; ++j) b[j] = lds_row8(Bs, (BN / 2) * wc + 16 * j + lr, lg);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m0 + 32 * wr + 16 * i + 4 * lg + q;
      if (m >= rows || !row_live(m, M, stack)) continue;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int n = n0 + (BN / 2) * wc + 16 * j + lr;
        if (n < N) ep(m, n, acc[i][j][q]);
      }
    }
}

template <class ALA, class ALB>
__global__ void __launch_bounds__(256) k_wgrad_bf16(RowRange rr, int stack, int N, int K, int rows_per_slice,
                                                    ALA A, ALB Bl, float* __restrict__ partial) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int rows = stack ? 2 * stack : M;
  const int n0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
  const int slice = blockIdx.z;
  const int r0 = slice * rows_per_slice;
  const int r1 = min(rows, r0 + rows_per_slice);
  constexpr int MS = 32;  // rows (the reduction index) per stage
  __shared__ __attribute__((aligned(16))) __bf16 As[64 * kBfRow];   // [n][m]
  __shared__ __attribute__((aligned(16))) __bf16 Bs[64 * kBfRow];   // [k][m]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, wr = wv >> 1, wc = wv & 1;
  const int lr = lane & 15, lg = lane >> 4;
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  // every thread stages rows 8 (tid / 64) .. + 7 of column tid % 64 (lanes
  // along the columns: coalesced loads) and writes each group of 8 to LDS
  // as one 16-byte store
  float ra[8], rb[8];
  const int sc = tid & 63, smq = 8 * (tid >> 6);
  auto fetch = [&](int m0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int m = m0 + smq + q;
      const bool live = m < r1 && row_live(m, M, stack);
      ra[q] = (live && n0 + sc < N) ? A(m, n0 + sc) : 0.0f;
      rb[q] = (live && k0 + sc < K) ? Bl(m, k0 + sc) : 0.0f;
    }
  };
  if (r0 < r1) fetch(r0);
  for (int m0 = r0; m0 < r1; m0 += MS) {
    {
      bf16x8_t va, vb;
#pragma unroll
      for (int q = 0; q < 8; ++q) { va[q] = (__bf16)ra[q]; vb[q] = (__bf16)rb[q]; }
      *reinterpret_cast<bf16x8_t*>(As + sc * kBfRow + smq) = va;
      *reinterpret_cast<bf16x8_t*>(Bs + sc * kBfRow + smq) = vb;
    }
    __syncthreads();
    if (m0 + MS < r1) fetch(m0 + MS);
    bf16x8_t a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = lds_row8(As, 32 * wr + 16 * i + lr, lg);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = lds_row8(Bs, 32 * wc + 16 * j + lr, lg);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
    __syncthreads();
  }
  float* P = partial + (int64_t)slice * N * K;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = n0 + 32 * wr + 16 * i + 4 * lg + q;
      if (n >= N) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int k = k0 + 32 * wc + 16 * j + lr;
        if (k < K) P[(int64_t)n * K + k] = acc[i][j][q];
      }
    }
}

// the second-order GEMM: BF16 MFMA for BF16 models, FP32 MFMA otherwise
template <bool NT, class AL, class EP>
inline void sgemm_so(bool bf16, hipStream_t st, RowRange rr, int64_t max_rows, int K, int N, const float* W, int ldw,
                     AL al, EP ep, int stack) {
  const int64_t rows = stack ? 2 * (int64_t)stack : max_rows;
  dim3 grid((unsigned)((rows + 63) / 64 > 0 ? (rows + 63) / 64 : 1), (unsigned)((N + 63) / 64));
  if (bf16 && N > 64) {
    grid.y = (unsigned)((N + 127) / 128);
    hipLaunchKernelGGL((k_sgemm_bf16<NT, 128, AL, EP>), grid, dim3(256), 0, st, rr, K, N, W, ldw, al, ep, stack);
  } else if (bf16)
    hipLaunchKernelGGL((k_sgemm_bf16<NT, 64, AL, EP>), grid, dim3(256), 0, st, rr, K, N, W, ldw, al, ep, stack);
  else
    hipLaunchKernelGGL((k_sgemm_mfma<NT, AL, EP>), grid, dim3(256), 0, st, rr, K, N, W, ldw, al, ep, stack);
}

}  // namespace afm
