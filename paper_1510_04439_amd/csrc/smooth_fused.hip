// Fused covariance smoother for d = 2 (placeholder until the fused kernels land).
#include "common.hpp"

namespace fpca {
bool smooth_cov_fused_d2_supported(const fpca_grid *, const double *) { return false; }
int smooth_cov_fused_d2(fpca_context *, const fpca_grid *, const float *, const float *, const double *, float *,
                        int8_t *, bool) {
  return set_error(FPCA_ERR_UNSUPPORTED, "fused d=2 smoother not built");
}
}  // namespace fpca
