// Step-kernel instantiations for u_s element type complex64, FP64 residual.
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(c64, cx<float>, false)
}  // namespace gadi
