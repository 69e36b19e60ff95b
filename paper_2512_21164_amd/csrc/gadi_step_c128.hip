// Step-kernel instantiations for u_s element type cx<double>.
#include "gadi_step.inc"

namespace gadi {
hipError_t launch_step_c128(int dim, int ry, const StepArgs& args, int grid, hipStream_t st) {
  return launch_step_dim<cx<double>>(dim, ry, args, grid, st);
}
int occupancy_c128(int dim, int ry) { return occupancy_dim<cx<double>>(dim, ry); }
}  // namespace gadi
