// Small utility kernels and the step-launch dispatch.
#include "gadi_step.inc"

namespace gadi {

#define GADI_DECLARE_STEP(NAME)                                                                      \
  hipError_t launch_step_##NAME(int dim, int ry, const StepArgs& args, int grid, hipStream_t st); \
  int occupancy_##NAME(int dim, int ry);
GADI_DECLARE_STEP(f64) GADI_DECLARE_STEP(f32) GADI_DECLARE_STEP(bf16)
GADI_DECLARE_STEP(c128) GADI_DECLARE_STEP(c64) GADI_DECLARE_STEP(cbf16)
GADI_DECLARE_STEP(f64_xr) GADI_DECLARE_STEP(f32_xr) GADI_DECLARE_STEP(bf16_xr)
GADI_DECLARE_STEP(c128_xr) GADI_DECLARE_STEP(c64_xr) GADI_DECLARE_STEP(cbf16_xr)
#undef GADI_DECLARE_STEP

int step_blocks_per_cu(int us, int cplx, int dim, int ry, int xr) {
  if (us < US_F64 || us > US_BF16) return 0;
  switch ((cplx ? 3 : 0) + us + (xr ? 6 : 0)) {
    case 0: return occupancy_f64(dim, ry);
    case 1: return occupancy_f32(dim, ry);
    case 2: return occupancy_bf16(dim, ry);
    case 3: return occupancy_c128(dim, ry);
    case 4: return occupancy_c64(dim, ry);
    case 5: return occupancy_cbf16(dim, ry);
    case 6: return occupancy_f64_xr(dim, ry);
    case 7: return occupancy_f32_xr(dim, ry);
    case 8: return occupancy_bf16_xr(dim, ry);
    case 9: return occupancy_c128_xr(dim, ry);
    case 10: return occupancy_c64_xr(dim, ry);
    case 11: return occupancy_cbf16_xr(dim, ry);
  }
  return 0;
}

hipError_t launch_step(int us, int cplx, int dim, int ry, int xr, const StepArgs& args, int grid, hipStream_t st) {
  if (us < US_F64 || us > US_BF16) return hipErrorInvalidValue;
  switch ((cplx ? 3 : 0) + us + (xr ? 6 : 0)) {
    case 0: return launch_step_f64(dim, ry, args, grid, st);
    case 1: return launch_step_f32(dim, ry, args, grid, st);
    case 2: return launch_step_bf16(dim, ry, args, grid, st);
    case 3: return launch_step_c128(dim, ry, args, grid, st);
    case 4: return launch_step_c64(dim, ry, args, grid, st);
    case 5: return launch_step_cbf16(dim, ry, args, grid, st);
    case 6: return launch_step_f64_xr(dim, ry, args, grid, st);
    case 7: return launch_step_f32_xr(dim, ry, args, grid, st);
    case 8: return launch_step_bf16_xr(dim, ry, args, grid, st);
    case 9: return launch_step_c128_xr(dim, ry, args, grid, st);
    case 10: return launch_step_c64_xr(dim, ry, args, grid, st);
    case 11: return launch_step_cbf16_xr(dim, ry, args, grid, st);
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

// r = b - A x at every unknown, one thread each: in FP64 (XR false, the
// stencil order of the step kernel) or with Dot2 sums (XR true, the same
// arithmetic as the outer phase's extra-precision residual).
template <bool CPLX, bool XR>
__global__ __launch_bounds__(256) void gadi_residual_dense(int dim, int nx, int ny, int nz, ACoef k,
                                                           const double* __restrict__ bin,
                                                           const double* __restrict__ xin,
                                                           double* __restrict__ rout) {
  using W = typename Wide<CPLX>::W;
  const W* x = reinterpret_cast<const W*>(xin);
  const W* b = reinterpret_cast<const W*>(bin);
  W* r = reinterpret_cast<W*>(rout);
  const int64_t n = (int64_t)nx * ny * nz;
  const int64_t pl = (int64_t)nx * ny;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ix = (int)(i % nx);
    const int64_t t = i / nx;
    const int iy = (int)(t % ny);
    const int iz = (int)(t / ny);
    Nbr<W> v;
    v.c = x[i];
    v.xm = ix > 0 ? x[i - 1] : W{};
    v.xp = ix < nx - 1 ? x[i + 1] : W{};
    if (dim == 2) {          // marching axis y
      v.ym = W{}; v.yp = W{};
      v.zm = iy > 0 ? x[i - nx] : W{};
      v.zp = iy < ny - 1 ? x[i + nx] : W{};
    } else {
      v.ym = iy > 0 ? x[i - nx] : W{};
      v.yp = iy < ny - 1 ? x[i + nx] : W{};
      v.zm = iz > 0 ? x[i - pl] : W{};
      v.zp = iz < nz - 1 ? x[i + pl] : W{};
    }
    W o;
    if constexpr (XR) {
      o = dim == 2 ? dot2_A<2>(k, v).residual(b[i]) : dot2_A<3>(k, v).residual(b[i]);
    } else {
      W a = k.c * v.c;
      a = a + k.lo[0] * v.xm + k.hi[0] * v.xp + k.lo[2] * v.zm + k.hi[2] * v.zp;
      if (dim == 3) a = a + k.lo[1] * v.ym + k.hi[1] * v.yp;
      a = ShiftOp<W>::add(a, v.c, k.sh);
      o = b[i] - a;
    }
    r[i] = o;
  }
}

hipError_t launch_residual_dense(int cplx, int xr, int dim, int nx, int ny, int nz, double center, const double* lo,
                                 const double* hi, double shift, const double* b, const double* x, double* r,
                                 hipStream_t st) {
  // kernel axis order: 0 = x, 1 = in-plane y (3D), 2 = marching axis (2D: y, 3D: z)
  ACoef k;
  k.c = center; k.sh = cplx ? shift : 0.0;
  k.lo[0] = lo[0]; k.hi[0] = hi[0];
  if (dim == 2) { k.lo[1] = 0.0; k.hi[1] = 0.0; k.lo[2] = lo[1]; k.hi[2] = hi[1]; }
  else { k.lo[1] = lo[1]; k.hi[1] = hi[1]; k.lo[2] = lo[2]; k.hi[2] = hi[2]; }
  const int64_t n = (int64_t)nx * ny * nz;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  const dim3 g((unsigned)blocks), bl(256);
  if (cplx) {
    if (xr) hipLaunchKernelGGL((gadi_residual_dense<true, true>), g, bl, 0, st, dim, nx, ny, nz, k, b, x, r);
    else hipLaunchKernelGGL((gadi_residual_dense<true, false>), g, bl, 0, st, dim, nx, ny, nz, k, b, x, r);
  } else {
    if (xr) hipLaunchKernelGGL((gadi_residual_dense<false, true>), g, bl, 0, st, dim, nx, ny, nz, k, b, x, r);
    else hipLaunchKernelGGL((gadi_residual_dense<false, false>), g, bl, 0, st, dim, nx, ny, nz, k, b, x, r);
  }
  return hipGetLastError();
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
