// Adam update of a flat parameter vector (Model Training: the parameters
// are optimised with Adam).  One thread per parameter, float64 moments.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device_util.h"
#include "internal.h"

namespace afm {

__global__ void k_adam(double* __restrict__ theta, const float* __restrict__ grad, double* __restrict__ m1,
                       double* __restrict__ m2, int64_t n, double lr, double b1, double b2, double eps, double c1,
                       double c2) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const double g = (double)grad[q];
    const double a = b1 * m1[q] + (1.0 - b1) * g;
    const double b = b2 * m2[q] + (1.0 - b2) * g * g;
    m1[q] = a;
    m2[q] = b;
    theta[q] -= lr * (a / c1) / (sqrt(b / c2) + eps);
  }
}

}  // namespace afm

extern "C" int afm_adam_step(double* theta, const float* grad, double* m1, double* m2, int64_t n, double lr,
                             double beta1, double beta2, double eps, int64_t t, void* stream) {
  using namespace afm;
  if (n < 0 || (n > 0 && (!theta || !grad || !m1 || !m2))) { set_error("null argument"); return AFM_E_INVALID; }
  if (t < 1 || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0) || !isfinite(lr)) {
    set_error("bad Adam parameters");
    return AFM_E_INVALID;
  }
  if (n == 0) return AFM_OK;
  const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 256, 4096)), dim3(256), 0, (hipStream_t)stream, theta, grad, m1, m2, n,
                     lr, beta1, beta2, eps, c1, c2);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}
