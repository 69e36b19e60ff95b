// Step-kernel instantiations for u_s element type float.
#include "gadi_step.inc"

namespace gadi {
hipError_t launch_step_f32(int dim, int ry, const StepArgs& args, int grid, hipStream_t st) {
  return launch_step_dim<float>(dim, ry, args, grid, st);
}
int occupancy_f32(int dim, int ry) { return occupancy_dim<float>(dim, ry); }
}  // namespace gadi
