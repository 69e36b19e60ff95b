// Internal layout shared by the host runtime and the gfx950 kernels.
//
// Each system (one A x = b) owns, inside its workspace:
//   GadiDesc   read-only description: grid, tiling, stencil coefficients,
//              parameters and buffer addresses (written by the host);
//   GadiCtl    the device-side state machine of Algorithm 1 (Section 2.3):
//              phase, iteration counters and the CG / CGNE scalars; only the
//              last tile of a step writes it;
//   partials   four doubles per tile for the reductions of a step;
//   counters   two-level tickets of the tiles finished in the current step
//              (last-tile detection);
//   history    per sweep: BE, relres, CG and CGNE iteration counts;
//   vectors    x^(k) (two FP64 buffers, ping-pong), padded b, and four
//              u_s vectors shared by the two inner solves.
// Vectors use a padded layout: element (i, j, k) at i + P*(j + ny*k) with the
// row pitch P = nx rounded up to 8 elements, so every 16-byte vector access
// of a row is aligned; the padding stays zero.
#pragma once
#include <stdint.h>

// BF16 elements per lane in the inner phases of real problems: 8 gives
// 16-byte lane accesses (7-8% faster 3D phases than 8-byte ones with 4, the
// same in 2D), at the cost of registers
#ifndef GADI_BF16_V
#define GADI_BF16_V 8
#endif

#ifndef GADI_TICKET_GROUPS
#define GADI_TICKET_GROUPS 16
#endif
// bytes of the ticket counters of one system: a top counter and
// GADI_TICKET_GROUPS group counters, 256 bytes apart
#define GADI_TICKET_BYTES (256 * (1 + GADI_TICKET_GROUPS))

namespace gadi {

enum Phase : int32_t {
  PH_IDLE = 0,
  PH_NORM_A = 1,   // t = A (v / ||v||)          power iteration on A^H A
  PH_NORM_AT = 2,  // v = A^H t
  PH_IMPORT = 3,   // b, x^(0): dense -> padded; ||b||
  PH_OUTER = 4,    // x^(k) = x^(k-1) + y^(k-1); r = b - A x^(k); norms; r -> u_s
  PH_H1 = 5,       // CG(H): p = r + beta p ; lazy z update ; (p, H p)
  PH_H2 = 6,       // CG(H): r -= a H p ; (r, r)
  PH_S0 = 7,       // CGNE(S) start: c = (2-omega) alpha z ; p = S^T c ; (c,c), (p,p)
  PH_S1 = 8,       // CGNE(S): p = S^T r + beta p ; lazy y update ; (p, p)
  PH_S2 = 9,       // CGNE(S): r -= a S p ; (r, r)
  PH_EXPORT = 10,  // x^(k) padded -> caller's dense x
  PH_DONE = 11,
  PH_ZFOLD = 12    // CG(H) ended after an even number of iterations: z += a_{j-2} p_{j-2}
};

enum Prec : int32_t { US_F64 = 0, US_F32 = 1, US_BF16 = 2 };

// Kernel classes whose CG updates z every second iteration with two terms:
// FP64 and FP32 (real), complex128, complex64 in 2D, and real BF16 in 3D with
// two or more rows per wave.  Measured on full-size fixed-iteration solves:
// the pairing made 2D complex64 4.7% faster (with one wave per SIMD less) and
// 3D BF16 with two rows 3.2% faster (same occupancy), but 2D BF16 1% and BF16
// pairs 5% slower (each losing a wave per SIMD), so those, 3D BF16 with one
// row and 3D complex64 (both would lose a wave per SIMD) update z every
// iteration.
__host__ __device__ constexpr bool pairs_z(int us, int cplx, int dim, int ry) {
  return us == US_F64 || (us == US_F32 && (!cplx || dim == 2)) || (us == US_BF16 && !cplx && dim == 3 && ry >= 2);
}

struct GadiCtl {
  int32_t phase;
  int32_t j;          // inner iteration index of the running CG / CGNE
  int32_t k;          // outer sweep whose residual PH_OUTER forms
  int32_t cur;        // x buffer holding x^(k)
  int32_t status;     // final status (GADI_OK ...)
  int32_t jH, jS;     // iterations of the last CG(H) and CGNE(S) solves
  int32_t k_ref;      // outer stagnation reference sweep
  int32_t jmin;       // inner stagnation reference iteration
  int32_t pS_base;    // direction buffer (1 or 2) holding CGNE direction p_0
  int32_t norm_it;    // power iterations left
  int32_t steps;      // non-idle steps executed (diagnostics)
  int64_t inner_h_total, inner_s_total;
  double be, relres, nr0, be_best, be_ref, normb, normA;
  double rho, rho0, a, beta, rho_min, a_prev, aH_last, aS_last;
  double norm_scale;  // 1/||v|| for the power iteration
  double a_pair[2];   // CG step size of iteration j in a_pair[j & 1] (z updated every second iteration)
  double pad1[1];
};

// Geometry of one tiling: V elements per lane, chunks of L planes along the
// marching axis (each tiling sized so that its wave tiles fill the device
// once); the in-plane row grouping is shared.
struct Tiling {
  int32_t V;
  int32_t nwx;        // wave tiles along x
  int32_t nwave;      // wave tiles in total
  int32_t ntiles;     // blocks of 4 waves
  int32_t L;          // planes per chunk
  int32_t nmc;        // chunks along the marching axis
  int32_t pad0, pad1;
};

struct GadiDesc {
  // problem
  int32_t dim, cplx, us, RY;
  int32_t nx, ny, nz, pad_n;
  int64_t P;           // padded row pitch (elements)
  int64_t n;           // nx * ny * nz
  int64_t nvec;        // elements per padded vector (P * ny * nz)
  // kernel geometry: axis 0 = x, axis 1 = in-plane y (3D only), axis 2 = marching
  int32_t ny_plane, nm;    // rows in a plane (3D: ny; 2D: 1), marching extent
  int32_t nwy, pad_g;      // row groups per plane
  int64_t sy, sm;          // strides (elements) of in-plane y and marching axes
  Tiling ti;               // inner phases: V = 16 bytes / sizeof(u_s element)
  Tiling to;               // FP64 phases: V = 16 bytes / sizeof(FP64 element)
  int32_t max_tiles, pad_t;
  // coefficients in kernel axis order
  double cA, shift_im, loA[3], hiA[3];
  double cH, mH[3];        // H = alpha I + M: centre, neighbour coefficient
  double alpha, nuS[3];    // S = alpha I + N: N(i, i+e) = +nu, N(i, i-e) = -nu
  double gamma;            // (2 - omega) alpha
  double g_re, g_im;       // complex problems: gamma / (alpha + i shift_im)
  float cAf, shift_imf, loAf[3], hiAf[3], cHf, mHf[3], alphaf, nuSf[3], gammaf, pad_f;
  // parameters
  double tol, div_factor, inner_tol_h, inner_tol_s;
  int64_t max_outer;
  int32_t stop_relres, stag_window, inner_stag, max_inner_h, max_inner_s, fixed_h, fixed_s;
  int32_t hist_len;
  // buffers
  double* xbuf[2];
  double* bpad;
  void* vs[4];             // u_s vectors: 0 = residual, 1,2 = directions, 3 = z (CG) / y (CGNE)
  const double* user_b;
  double* user_x;
  double* partials;        // 4 doubles per tile
  uint32_t* counter;       // top counter, followed by the group counters
  GadiCtl* ctl;
  double* hist;            // 4 doubles per sweep
};

// Table of systems advanced by one step launch (all of one kernel class).
struct BatchTable {
  int32_t nsys;
  int32_t total_tiles;     // sum over systems of max_tiles
  int32_t slots;           // total_tiles rounded up to a multiple of 8
  int32_t pad;
  GadiDesc** desc;         // [nsys]
  int32_t* tile_start;     // [nsys + 1] prefix sums of max_tiles
};

// Kernel argument of a step launch: the table, and for a table of one system
// that system's descriptor and control block (null otherwise), which saves
// the kernel two dependent loads before it knows its phase.
struct StepArgs {
  const BatchTable* tab;
  const GadiDesc* one;
  const GadiCtl* one_ctl;
};

// Host: record the message returned by gadi_last_error() and pass the status on
// (for the C-ABI entry points outside gadi_api.cpp).
int32_t set_error(int32_t status, const char* msg);

}  // namespace gadi
