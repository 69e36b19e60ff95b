// Step-kernel instantiations for u_s element type bf16.
#include "gadi_step.inc"

namespace gadi {
hipError_t launch_step_bf16(int dim, int ry, const StepArgs& args, int grid, hipStream_t st) {
  return launch_step_dim<bf16>(dim, ry, args, grid, st);
}
int occupancy_bf16(int dim, int ry) { return occupancy_dim<bf16>(dim, ry); }
}  // namespace gadi
