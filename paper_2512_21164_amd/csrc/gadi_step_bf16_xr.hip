// Step-kernel instantiations for u_s element type BF16 storage (FP32 arithmetic), residual in
// extra precision (Dot2 sums).
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(bf16_xr, bf16, true)
}  // namespace gadi
