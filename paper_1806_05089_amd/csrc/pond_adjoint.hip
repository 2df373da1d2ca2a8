// Adjoint (vector-Jacobian product) of the PonD step.
#include <hip/hip_runtime.h>

#include "pond_device.hpp"
#include "pond_internal.hpp"

namespace pond {

hipError_t launch_adjoint(const pond_config&, const void*, const double*, const uint8_t*,
                          const double*, const double*, double*, double*, double*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace pond
