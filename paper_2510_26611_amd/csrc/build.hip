// Rank reduction of the long-range sum on the device (Algorithm TEP step 4).
#include "internal.h"

namespace rsd {

rsd_status build_factors(Context* ctx, Tensor* t, const double* d_charges, const double* d_positions) {
  (void)ctx; (void)t; (void)d_charges; (void)d_positions;
  set_error("rsd_build_rs_tensor: device rank reduction not available in this build");
  return RSD_E_UNSUPPORTED;
}

}  // namespace rsd
