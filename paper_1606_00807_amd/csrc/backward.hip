// Reverse-mode derivative of fit + analysis (placeholder).
#include "device.h"

namespace enkfmc {
hipError_t launch_backward(enkfmc_plan *, const Dev &, const void *, int32_t, int64_t, const double *, const double *,
                           double, const double *, double *, double *, double *, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace enkfmc
