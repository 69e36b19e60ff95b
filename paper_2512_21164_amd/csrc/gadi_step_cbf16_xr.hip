// Step-kernel instantiations for u_s element type BF16 pairs (complex, FP32 arithmetic), residual in
// extra precision (Dot2 sums).
#include "gadi_step.inc"

namespace gadi {
GADI_STEP_INSTANCE(cbf16_xr, cx<bf16>, true)
}  // namespace gadi
