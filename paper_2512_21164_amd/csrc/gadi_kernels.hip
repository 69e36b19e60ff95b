// Small utility kernels and the step-launch dispatch.
#include "gadi_step.inc"

namespace gadi {

hipError_t launch_step_f64(int dim, int ry, const StepArgs& args, int grid, hipStream_t st);
hipError_t launch_step_f32(int dim, int ry, const StepArgs& args, int grid, hipStream_t st);
hipError_t launch_step_bf16(int dim, int ry, const StepArgs& args, int grid, hipStream_t st);
hipError_t launch_step_c128(int dim, int ry, const StepArgs& args, int grid, hipStream_t st);
hipError_t launch_step_c64(int dim, int ry, const StepArgs& args, int grid, hipStream_t st);
hipError_t launch_step_cbf16(int dim, int ry, const StepArgs& args, int grid, hipStream_t st);

int occupancy_f64(int dim, int ry);
int occupancy_f32(int dim, int ry);
int occupancy_bf16(int dim, int ry);
int occupancy_c128(int dim, int ry);
int occupancy_c64(int dim, int ry);
int occupancy_cbf16(int dim, int ry);

int step_blocks_per_cu(int us, int cplx, int dim, int ry) {
  if (!cplx) {
    switch (us) {
      case US_F64: return occupancy_f64(dim, ry);
      case US_F32: return occupancy_f32(dim, ry);
      case US_BF16: return occupancy_bf16(dim, ry);
    }
  } else {
    switch (us) {
      case US_F64: return occupancy_c128(dim, ry);
      case US_F32: return occupancy_c64(dim, ry);
      case US_BF16: return occupancy_cbf16(dim, ry);
    }
  }
  return 0;
}

hipError_t launch_step(int us, int cplx, int dim, int ry, const StepArgs& args, int grid, hipStream_t st) {
  if (!cplx) {
    switch (us) {
      case US_F64: return launch_step_f64(dim, ry, args, grid, st);
      case US_F32: return launch_step_f32(dim, ry, args, grid, st);
      case US_BF16: return launch_step_bf16(dim, ry, args, grid, st);
    }
  } else {
    switch (us) {
      case US_F64: return launch_step_c128(dim, ry, args, grid, st);
      case US_F32: return launch_step_c64(dim, ry, args, grid, st);
      case US_BF16: return launch_step_cbf16(dim, ry, args, grid, st);
    }
  }
  return hipErrorInvalidValue;
}

__global__ void gadi_set_phase(GadiCtl* c, int phase, int norm_iters, double norm_scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->phase = phase;
    if (phase == PH_NORM_A) { c->j = 0; c->norm_it = norm_iters; c->norm_scale = norm_scale; }
  }
}

__global__ void gadi_set_io(GadiDesc* d, const double* b, double* x) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { d->user_b = b; d->user_x = x; }
}

__global__ void gadi_set_norm(GadiCtl* c, double normA) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c->normA = normA;
}

// dense y = A x (or A^H x) for b = A x_true etc.; one thread per unknown
template <bool CPLX>
__global__ __launch_bounds__(256) void gadi_apply_dense(int dim, int nx, int ny, int nz, double cA, double lo0, double hi0,
                                                        double lo1, double hi1, double lo2, double hi2, double shift,
                                                        int transpose, const double* __restrict__ xin,
                                                        double* __restrict__ yout) {
  using W = typename Wide<CPLX>::W;
  const W* x = reinterpret_cast<const W*>(xin);
  W* y = reinterpret_cast<W*>(yout);
  const int64_t n = (int64_t)nx * ny * nz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ix = (int)(i % nx);
    const int64_t t = i / nx;
    const int iy = (int)(t % ny);
    const int iz = (int)(t / ny);
    double l0 = transpose ? hi0 : lo0, h0 = transpose ? lo0 : hi0;
    double l1 = transpose ? hi1 : lo1, h1 = transpose ? lo1 : hi1;
    double l2 = transpose ? hi2 : lo2, h2 = transpose ? lo2 : hi2;
    W o = cA * x[i];
    if (ix > 0) o = o + l0 * x[i - 1];
    if (ix < nx - 1) o = o + h0 * x[i + 1];
    if (iy > 0) o = o + l1 * x[i - nx];
    if (iy < ny - 1) o = o + h1 * x[i + nx];
    if (dim == 3) {
      const int64_t pl = (int64_t)nx * ny;
      if (iz > 0) o = o + l2 * x[i - pl];
      if (iz < nz - 1) o = o + h2 * x[i + pl];
    }
    o = ShiftOp<W>::add(o, x[i], transpose ? -shift : shift);
    y[i] = o;
  }
}

hipError_t launch_set_phase(GadiCtl* c, int phase, int norm_iters, double norm_scale, hipStream_t st) {
  hipLaunchKernelGGL(gadi_set_phase, dim3(1), dim3(64), 0, st, c, phase, norm_iters, norm_scale);
  return hipGetLastError();
}

hipError_t launch_set_io(GadiDesc* d, const double* b, double* x, hipStream_t st) {
  hipLaunchKernelGGL(gadi_set_io, dim3(1), dim3(64), 0, st, d, b, x);
  return hipGetLastError();
}

hipError_t launch_set_norm(GadiCtl* c, double normA, hipStream_t st) {
  hipLaunchKernelGGL(gadi_set_norm, dim3(1), dim3(64), 0, st, c, normA);
  return hipGetLastError();
}

hipError_t launch_apply_dense(int cplx, int dim, int nx, int ny, int nz, double cA, const double* lo, const double* hi,
                              double shift, int transpose, const double* x, double* y, hipStream_t st) {
  const int64_t n = (int64_t)nx * ny * nz;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (cplx)
    hipLaunchKernelGGL(gadi_apply_dense<true>, dim3((unsigned)blocks), dim3(256), 0, st, dim, nx, ny, nz, cA, lo[0],
                       hi[0], lo[1], hi[1], lo[2], hi[2], shift, transpose, x, y);
  else
    hipLaunchKernelGGL(gadi_apply_dense<false>, dim3((unsigned)blocks), dim3(256), 0, st, dim, nx, ny, nz, cA, lo[0],
                       hi[0], lo[1], hi[1], lo[2], hi[2], shift, transpose, x, y);
  return hipGetLastError();
}

}  // namespace gadi
