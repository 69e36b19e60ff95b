// Step-kernel instantiations for u_s element type cx<bf16>.
#include "gadi_step.inc"

namespace gadi {
hipError_t launch_step_cbf16(int dim, int ry, const StepArgs& args, int grid, hipStream_t st) {
  return launch_step_dim<cx<bf16>>(dim, ry, args, grid, st);
}
int occupancy_cbf16(int dim, int ry) { return occupancy_dim<cx<bf16>>(dim, ry); }
}  // namespace gadi
