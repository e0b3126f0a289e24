// Entry points whose device path is not built yet report HSS_ERR_UNSUPPORTED.
#include "hss_internal.h"

namespace hss {
void solve_fp32(hss_matrix_t, const double*, double*, int64_t, int64_t) {
  throw Error{HSS_ERR_UNSUPPORTED, "FP32 solve not available"};
}
}  // namespace hss

extern "C" {
hss_status hss_ulv_solve_refined(hss_ctx_t, hss_matrix_t, const double*, double*, int64_t, int64_t, double,
                                 int32_t, int32_t*, double*) {
  hss::set_error("refinement not available");
  return HSS_ERR_UNSUPPORTED;
}
}
