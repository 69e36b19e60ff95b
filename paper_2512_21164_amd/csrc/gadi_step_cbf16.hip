// Step-kernel instantiations for u_s element type BF16 pairs (complex, FP32 arithmetic), FP64 residual.
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(cbf16, cx<bf16>, false)
}  // namespace gadi
