// Edge vector of a listed edge, shared by the geometry kernel and the
// cutoff compaction so both take the same decision for |delta| < r_c:
//   delta = (r_j - r_i) + (n0 a + n1 b) + n2 c   (float64, rounded per
//   operation, no contraction), then float32 components and norm.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace afm {

__device__ __forceinline__ void edge_vec_f32(const double* __restrict__ pos, const double* __restrict__ cell,
                                             bool per, int64_t sl, int64_t i, int64_t j,
                                             const int8_t* __restrict__ sh, float& dx, float& dy, float& dz) {
  double d[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double s = 0.0;
    if (per) {
      const double* h = cell + 9 * sl;
      s = __dadd_rn(__dadd_rn(__dmul_rn((double)sh[0], h[q]), __dmul_rn((double)sh[1], h[3 + q])),
                    __dmul_rn((double)sh[2], h[6 + q]));
    }
    d[q] = __dadd_rn(__dsub_rn(pos[3 * j + q], pos[3 * i + q]), s);
  }
  dx = (float)d[0];
  dy = (float)d[1];
  dz = (float)d[2];
}

__device__ __forceinline__ float edge_norm_f32(float dx, float dy, float dz) {
  return sqrtf(__fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz)));
}

// structure of atom i (seg: [B+1] offsets)
__device__ __forceinline__ int64_t struct_of(const int64_t* __restrict__ seg, int64_t B, int64_t i) {
  int64_t lo = 0, hi = B;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (seg[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace afm
