// BF16 MFMA MLP chains (placeholder until the gfx950 kernels land).
#include <hip/hip_runtime.h>

#include <vector>

#include "gemm_f32.h"
#include "internal.h"

namespace afm {

int64_t bf16_frag_bytes(const afm_model*) { return 0; }
void pack_bf16_frags(const afm_model*, const std::vector<const double*>&, std::vector<char>& out, DevWeights*) {
  out.clear();
}
int mfma_twobody_fwd(const afm_model*, const afm_workspace*, const WsLayout&, RowRange, const int32_t*, hipStream_t) {
  set_error("BF16 MFMA path not built");
  return AFM_E_UNSUPPORTED;
}
int mfma_latent_fwd(const afm_model*, const afm_workspace*, const WsLayout&, RowRange, int, hipStream_t) {
  set_error("BF16 MFMA path not built");
  return AFM_E_UNSUPPORTED;
}
int mfma_latent_bwd(const afm_model*, const afm_workspace*, const WsLayout&, RowRange, int, const int32_t*,
                    const int64_t*, int64_t, const double*, hipStream_t) {
  set_error("BF16 MFMA path not built");
  return AFM_E_UNSUPPORTED;
}
int mfma_twobody_bwd(const afm_model*, const afm_workspace*, const WsLayout&, RowRange, const int32_t*, hipStream_t) {
  set_error("BF16 MFMA path not built");
  return AFM_E_UNSUPPORTED;
}

}  // namespace afm
