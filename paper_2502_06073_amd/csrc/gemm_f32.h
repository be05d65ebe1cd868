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

template <bool NT, class AL, class EP>
inline void sgemm(hipStream_t st, RowRange rr, int64_t max_rows, int K, int N, const float* W, int ldw, AL al,
                  EP ep, int stack = 0) {
  const int64_t rows = stack ? 2 * (int64_t)stack : max_rows;
  dim3 grid((unsigned)((rows + 63) / 64 > 0 ? (rows + 63) / 64 : 1), (unsigned)((N + 63) / 64));
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

}  // namespace afm
