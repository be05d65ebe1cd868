// Small device helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace afm {

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ __forceinline__ float silu_f(float a) { return a / (1.0f + expf(-a)); }

// silu'(a) = s (1 + a (1 - s)), s = sigmoid(a)
__device__ __forceinline__ float dsilu_f(float a) {
  const float s = 1.0f / (1.0f + expf(-a));
  return s * (1.0f + a * (1.0f - s));
}

// sum over groups of G consecutive lanes (G a power of two <= 64)
template <int G>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v);

// Zero `bytes` (multiple of 4) with a kernel (safe inside captured graphs).
int zero_async(void* p, int64_t bytes, hipStream_t st);

inline unsigned grid_for(int64_t n, int b, int64_t cap = 1 << 30) {
  int64_t g = (n + b - 1) / b;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Spherical harmonics (component normalised, no Condon-Shortley phase,
// l = 1 ordered (y, z, x)) of a unit vector, 9 values for l <= 2.
__device__ __forceinline__ void sh9(float x, float y, float z, float* Y) {
  const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s5h = 1.118033988749895f;
  Y[0] = 1.0f;
  Y[1] = s3 * y; Y[2] = s3 * z; Y[3] = s3 * x;
  Y[4] = s15 * x * y; Y[5] = s15 * y * z; Y[6] = s5h * (3.0f * z * z - 1.0f);
  Y[7] = s15 * x * z; Y[8] = 0.5f * s15 * (x * x - y * y);
}

// d Y_k / d(x, y, z) for the polynomial forms above (before projection
// onto the sphere's tangent plane).
__device__ __forceinline__ void sh9_grad(float x, float y, float z, const float* gY, float* gu) {
  const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s5h = 1.118033988749895f;
  float gx = 0, gy = 0, gz = 0;
  gy += s3 * gY[1]; gz += s3 * gY[2]; gx += s3 * gY[3];
  gx += s15 * y * gY[4]; gy += s15 * x * gY[4];
  gy += s15 * z * gY[5]; gz += s15 * y * gY[5];
  gz += s5h * 6.0f * z * gY[6];
  gx += s15 * z * gY[7]; gz += s15 * x * gY[7];
  gx += s15 * x * gY[8]; gy -= s15 * y * gY[8];
  gu[0] = gx; gu[1] = gy; gu[2] = gz;
}

}  // namespace afm
