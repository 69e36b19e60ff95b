// Step-kernel instantiations for u_s element type complex128, FP64 residual.
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(c128, cx<double>, false)
}  // namespace gadi
