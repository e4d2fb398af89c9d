#include <hip/hip_runtime.h>
#include "rjsmc_internal.h"
namespace rjsmc {
hipError_t launch_loglik_grad(const DevSystem &, const DevParticles &, int, int, const double *, double *,
                              const DevGrad &, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace rjsmc
