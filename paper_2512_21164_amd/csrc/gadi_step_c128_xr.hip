// Step-kernel instantiations for u_s element type complex128, residual in
// extra precision (Dot2 sums).
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(c128_xr, cx<double>, true)
}  // namespace gadi
