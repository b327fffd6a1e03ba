// Instantiations of the stage and time-step kernels for one equation and
// dimension (one translation unit each so they build in parallel).
#include "stage_kernel.hpp"

namespace idp {
IDP_DEFINE_LAUNCHERS(advv2, EQ_ADVV, 2)
}  // namespace idp
