// FP32 GEMM on the vector ALUs for the plain-FP32 path:
//   C[m][n] = sum_k A(m, k) * B(k, n),   m < rows of the current chunk
// with A read through a loader functor (concatenations, SiLU on load), B a
// row-major weight matrix used as W^T ([N][K], "NT") or W ([K][N], "NN"), and
// a fused epilogue functor.  64 x 64 tiles, K steps of 16 staged in LDS,
// 4 x 4 outputs per thread.
#pragma once
#include <hip/hip_runtime.h>

#include "edge_layout.h"

namespace afm {

template <bool NT, class AL, class EP>
__global__ void __launch_bounds__(256) k_sgemm(RowRange rr, int K, int N, const float* __restrict__ W,
                                               int ldw, AL al, EP ep) {
  int64_t e0, e1;
  rr.get(e0, e1);
  const int M = (int)(e1 - e0);
  const int m0 = blockIdx.x * 64;
  if (m0 >= M) return;
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
      As[kk][r] = (m < M && k < K) ? al(m, k) : 0.0f;
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
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n < N) ep(m, n, acc[i][j]);
    }
  }
}

template <bool NT, class AL, class EP>
inline void sgemm(hipStream_t st, RowRange rr, int64_t max_rows, int K, int N, const float* W, int ldw,
                  AL al, EP ep) {
  dim3 grid((unsigned)((max_rows + 63) / 64 > 0 ? (max_rows + 63) / 64 : 1), (unsigned)((N + 63) / 64));
  hipLaunchKernelGGL((k_sgemm<NT, AL, EP>), grid, dim3(256), 0, st, rr, K, N, W, ldw, al, ep);
}

}  // namespace afm
