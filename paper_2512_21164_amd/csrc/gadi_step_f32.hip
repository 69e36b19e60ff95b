// Step-kernel instantiations for u_s element type float, FP64 residual.
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(f32, float, false)
}  // namespace gadi
