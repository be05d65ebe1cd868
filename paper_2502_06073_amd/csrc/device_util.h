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

// Sums of up to 16 values over the 64 lanes of a wavefront, as a
// reduce-scatter: each exchange step halves the values a lane carries, so 16
// sums cost 8 + 4 cross-row swaps (v_permlane32/16_swap) and 3 in-row DPP
// steps instead of 16 x 6 cross-lane shuffles.  On return, lane l holds the
// total of value (l >> 2) (lanes 4k..4k+3 all hold value k).
__device__ __forceinline__ float dpp_f(float v, int ctrl_id) {
  const int x = __builtin_bit_cast(int, v);
  int r;
  switch (ctrl_id) {  // dpp_ctrl must be an immediate
    case 0: r = __builtin_amdgcn_update_dpp(0, x, 0x140, 0xf, 0xf, false); break;  // row_mirror (l <-> 15-l)
    case 1: r = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xf, 0xf, false); break;  // row_half_mirror (l <-> 7-l)
    case 2: r = __builtin_amdgcn_update_dpp(0, x, 0x4e, 0xf, 0xf, false); break;   // quad_perm [2,3,0,1]
    default: r = __builtin_amdgcn_update_dpp(0, x, 0xb1, 0xf, 0xf, false); break;  // quad_perm [1,0,3,2]
  }
  return __builtin_bit_cast(float, r);
}

__device__ __forceinline__ float wave_sum16(float (&v)[16], int lane) {
  // lanes [0,32) end up with values 0..7, lanes [32,64) with 8..15
  float u[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(int, v[k]), __builtin_bit_cast(int, v[k + 8]),
                                                    false, false);
    u[k] = __builtin_bit_cast(float, (int)r[0]) + __builtin_bit_cast(float, (int)r[1]);
  }
  // even rows of 16 keep 0..3 (of the eight), odd rows 4..7
  float w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(int, u[k]), __builtin_bit_cast(int, u[k + 4]),
                                                    false, false);
    w[k] = __builtin_bit_cast(float, (int)r[0]) + __builtin_bit_cast(float, (int)r[1]);
  }
  // in-row halves (partner l <-> 15 - l differs in bit 3): keep 0,1 or 2,3
  const bool b3 = lane & 8, b2 = lane & 4;
  float x[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float keep = b3 ? w[k + 2] : w[k], send = b3 ? w[k] : w[k + 2];
    x[k] = keep + dpp_f(send, 0);
  }
  // quarter rows (partner l <-> 7 - l within 8 lanes differs in bit 2)
  const float keep = b2 ? x[1] : x[0], send = b2 ? x[0] : x[1];
  float y = keep + dpp_f(send, 1);
  y += dpp_f(y, 2);
  y += dpp_f(y, 3);
  return y;
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

// Y^3 (m = -3..3, no Condon-Shortley phase, sum_m Y^2 = 7 on the sphere),
// written with x^2 + y^2 + z^2 = 1 substituted; the gradient of these
// polynomial forms differs from the homogeneous ones only radially, which
// the tangent-plane projection of the caller removes.
__device__ __forceinline__ void sh_l3(float x, float y, float z, float* Y) {
  const float a3 = 2.091650066335189f, a2 = 10.246950765959598f, a1 = 1.620185174601965f,
              a0 = 1.3228756555322954f;
  Y[0] = a3 * y * (3.0f * x * x - y * y);
  Y[1] = a2 * x * y * z;
  Y[2] = a1 * y * (5.0f * z * z - 1.0f);
  Y[3] = a0 * z * (5.0f * z * z - 3.0f);
  Y[4] = a1 * x * (5.0f * z * z - 1.0f);
  Y[5] = 0.5f * a2 * z * (x * x - y * y);
  Y[6] = a3 * x * (x * x - 3.0f * y * y);
}
// gu += sum_k gY[k] dY^3_k / d(x, y, z)
__device__ __forceinline__ void sh_l3_grad(float x, float y, float z, const float* gY, float* gu) {
  const float a3 = 2.091650066335189f, a2 = 10.246950765959598f, a1 = 1.620185174601965f,
              a0 = 1.3228756555322954f;
  float gx = 0, gy = 0, gz = 0;
  gx += a3 * 6.0f * x * y * gY[0];            gy += a3 * 3.0f * (x * x - y * y) * gY[0];
  gx += a2 * y * z * gY[1];                   gy += a2 * x * z * gY[1];               gz += a2 * x * y * gY[1];
  gy += a1 * (5.0f * z * z - 1.0f) * gY[2];   gz += a1 * 10.0f * y * z * gY[2];
  gz += a0 * (15.0f * z * z - 3.0f) * gY[3];
  gx += a1 * (5.0f * z * z - 1.0f) * gY[4];   gz += a1 * 10.0f * x * z * gY[4];
  gx += a2 * x * z * gY[5];                   gy -= a2 * y * z * gY[5];               gz += 0.5f * a2 * (x * x - y * y) * gY[5];
  gx += a3 * 3.0f * (x * x - y * y) * gY[6];  gy -= a3 * 6.0f * x * y * gY[6];
  gu[0] += gx; gu[1] += gy; gu[2] += gz;
}

}  // namespace afm
