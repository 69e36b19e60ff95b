// Step-kernel instantiations for u_s element type double.
#include "gadi_step.inc"

namespace gadi {
hipError_t launch_step_f64(int dim, int ry, const StepArgs& args, int grid, hipStream_t st) {
  return launch_step_dim<double>(dim, ry, args, grid, st);
}
int occupancy_f64(int dim, int ry) { return occupancy_dim<double>(dim, ry); }
}  // namespace gadi
