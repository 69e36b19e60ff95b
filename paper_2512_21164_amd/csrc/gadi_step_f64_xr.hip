// Step-kernel instantiations for u_s element type float64, residual in
// extra precision (Dot2 sums).
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(f64_xr, double, true)
}  // namespace gadi
