// Step-kernel instantiations for u_s element type float, residual in
// extra precision (Dot2 sums).
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(f32_xr, float, true)
}  // namespace gadi
