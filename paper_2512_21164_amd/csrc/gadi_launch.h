// Host-callable launchers of the gfx950 kernels (defined in gadi_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "gadi_internal.h"

namespace gadi {

// One device step for every system of `tab` (all of class us/cplx/dim/ry/xr;
// xr selects the kernels with the extra-precision residual).
hipError_t launch_step(int us, int cplx, int dim, int ry, int xr, const StepArgs& args, int grid, hipStream_t st);
// Resident 256-thread blocks per CU of the step kernel of this class (0 if unknown).
int step_blocks_per_cu(int us, int cplx, int dim, int ry, int xr);
hipError_t launch_set_phase(GadiCtl* c, int phase, int norm_iters, double norm_scale, hipStream_t st);
hipError_t launch_set_io(GadiDesc* d, const double* b, double* x, hipStream_t st);
hipError_t launch_set_norm(GadiCtl* c, double normA, hipStream_t st);
hipError_t launch_apply_dense(int cplx, int dim, int nx, int ny, int nz, double cA, const double* lo, const double* hi,
                              double shift, int transpose, const double* x, double* y, hipStream_t st);
// r = b - A x (dense vectors), FP64 (xr = 0) or extra precision (xr = 1).
hipError_t launch_residual_dense(int cplx, int xr, int dim, int nx, int ny, int nz, double center, const double* lo,
                                 const double* hi, double shift, const double* b, const double* x, double* r,
                                 hipStream_t st);

}  // namespace gadi
