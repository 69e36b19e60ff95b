// Step-kernel instantiations for u_s element type complex64, residual in
// extra precision (Dot2 sums).
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(c64_xr, cx<float>, true)
}  // namespace gadi
