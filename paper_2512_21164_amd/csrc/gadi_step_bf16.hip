// Step-kernel instantiations for u_s element type BF16 storage (FP32 arithmetic), FP64 residual.
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(bf16, bf16, false)
}  // namespace gadi
