// Placeholder until the adjoint kernel lands.
#include <hip/hip_runtime.h>

#include "dg_launch.hpp"

namespace tetdg {
hipError_t launch_vjp(int, int, const VjpArgs&, hipStream_t) { return hipErrorNotSupported; }
}  // namespace tetdg
