// Batched FP64 fit (placeholder until the wavefront kernel lands): routes to
// the plain kernel so the entry point is defined.
#include "device.h"

namespace enkfmc {
hipError_t launch_fit_batched(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s) {
  return launch_fit_plain(p, d, lam, s);
}
}  // namespace enkfmc
