// Step-kernel instantiations for u_s element type cx<float>.
#include "gadi_step.inc"

namespace gadi {
hipError_t launch_step_c64(int dim, int ry, const StepArgs& args, int grid, hipStream_t st) {
  return launch_step_dim<cx<float>>(dim, ry, args, grid, st);
}
int occupancy_c64(int dim, int ry) { return occupancy_dim<cx<float>>(dim, ry); }
}  // namespace gadi
