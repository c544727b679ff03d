// Adjoint kernels (placeholder until the reverse sweep lands).
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace selinv {

hipError_t launch_backward(const DevPlan &, const DevPlan *, const LaunchAux &, const void *, const void *,
                           const void *, void *, void *, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace selinv
