// Adjoint (transposed) operator and gradients -- filled in below.
#include "device_util.h"

namespace pbtc {

int apply_transpose(pbtc_plan& pl, hipStream_t, const double*, double*, int, int) {
  pl.err = "transposed operator not available in this build";
  return PBTC_EINVAL;
}

int device_backward(pbtc_plan& pl, hipStream_t, double, double*, double*, double*, pbtc_result*) {
  pl.err = "backward not available in this build";
  return PBTC_EINVAL;
}

int device_solve_batch(pbtc_plan**, int, hipStream_t, pbtc_result*) { return PBTC_EINVAL; }

}  // namespace pbtc
