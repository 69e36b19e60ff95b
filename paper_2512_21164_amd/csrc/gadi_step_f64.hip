// Step-kernel instantiations for u_s element type float64, FP64 residual.
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(f64, double, false)
}  // namespace gadi
