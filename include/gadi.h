/*
 * gadi.h -- C ABI of the MI355X (gfx950) implementation of mixed-precision
 * GADI (general alternating-direction implicit iteration) for A x = b.
 *
 * Method (arXiv 2512.21164):
 *   splitting   A = M + N, H = alpha I + M, S = alpha I + N       eq. (split), Section 3.1
 *               with the Hermitian / skew-Hermitian choice
 *               M = (A + A^H)/2, N = (A - A^H)/2                  Sections 5.2-5.4
 *   iteration   Algorithm 1 (Section 2.3): from x^(0),
 *                 r = b - A x           in u_r  (FP64, or FP64 pairs: GADI_F64X2)
 *                 solve H z = r         in u_s  (CG, Section 5.1)
 *                 solve S y = (2-omega) alpha z   in u_s  (CG on the normal equations)
 *                 x = x + y             in u    (FP64 here)
 *   stopping    backward error ||b - A x|| / (||A|| ||x|| + ||b||) <= tol
 *               (Section 3, 2-norms), or the relative residual ||r||/||r0||
 *               that the experiments of Section 5 use.
 *
 * The operator A is matrix-free: a 5-point (2D) or 7-point (3D) constant
 * coefficient stencil on the interior of a grid with zero Dirichlet values
 * outside it (gadi_stencil).  Complex problems (Section 5.4) add a constant
 * imaginary diagonal shift: A = L + i*shift_im*I.
 *
 * Memory.  The library never allocates device memory.  Every buffer is owned
 * by the caller: the workspace (size from gadi_workspace_bytes), b and x.
 * Device pointers are plain device addresses (e.g. torch tensor data_ptr()).
 * Vectors are dense, x-fastest: index = i + nx*(j + ny*k).  Real problems use
 * float64; complex problems use interleaved complex128 (re, im).
 * Streams are hipStream_t passed as void* (NULL = default stream).  A handle
 * is bound to one stream and is not thread-safe; calls on one handle must not
 * overlap.
 *
 * Errors.  Functions return a gadi_status.  Negative values are errors and
 * leave the handle usable (argument errors are detected before any device
 * work).  GADI_ERR_HIP carries the HIP error text in gadi_last_error().
 * Positive values are numerical outcomes of a finished solve.
 */
#ifndef GADI_H
#define GADI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gadi_status;

enum {
  GADI_OK = 0,              /* converged: criterion <= tol                         */
  GADI_NOT_CONVERGED = 1,   /* reached max_outer sweeps                            */
  GADI_STAGNATED = 2,       /* BE did not drop below 0.99x its reference in
                               stag_window sweeps (Section 4.3, step 3)            */
  GADI_DIVERGED = 3,        /* BE not finite, or above div_factor * best BE        */
  GADI_RUNNING = 4,         /* asynchronous solve still in progress                */
  GADI_ERR_INVALID_ARG = -1,
  GADI_ERR_UNSUPPORTED = -2,
  GADI_ERR_WORKSPACE = -3,  /* workspace missing, misaligned or too small          */
  GADI_ERR_HIP = -4,
  GADI_ERR_CAPACITY = -5,   /* batch full, or budget exceeded                      */
  GADI_ERR_STATE = -6       /* call not valid in the handle's current state        */
};

/* Precision of a stage of Algorithm 1 (u_r, u, u_s; Section 2.3, Table 1).
 * GADI_BF16 means BF16 storage with FP32 arithmetic (Section 5.1).
 * GADI_F64X2 (u_r only) is the extra-precision residual u_r < u of Section
 * 2.3: FP64 data, products and sums carried exactly as unevaluated pairs of
 * FP64 numbers (FMA TwoProduct, TwoSum; the Dot2 scheme of Ogita, Rump and
 * Oishi, 2005), so that r = b - A x is as accurate as if computed in twice
 * the FP64 precision and rounded once to FP64:
 *   |r_i - (b - A x)_i| <= 2^-53 |(b - A x)_i| + gamma_K^2 sum_j |a_ij x_j|,
 * gamma_K = K 2^-53 / (1 - K 2^-53), K the terms of row i (6 to 9).  This
 * removes the kappa(A) u_r term from the forward-error limit (Theorem 2). */
typedef enum { GADI_F64 = 0, GADI_F32 = 1, GADI_BF16 = 2, GADI_F64X2 = 3 } gadi_prec;

/* The operator A (matrix-free).  At interior grid point p:
 *   (A u)_p = center*u_p + sum_d ( lo[d]*u_{p-e_d} + hi[d]*u_{p+e_d} )
 *             + i*shift_im*u_p                          (is_complex only)
 * with u = 0 outside the grid.  2D: dim = 2, n[2] = 1, lo[2] = hi[2] = 0.
 * Complex problems must have a symmetric real part (lo[d] == hi[d]) so that
 * N = i*shift_im*I and the S solve is pointwise (Section 5.4's problem class);
 * otherwise GADI_ERR_UNSUPPORTED. */
typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t is_complex;   /* 0 real float64; 1 complex128 interleaved */
  int64_t n[3];         /* interior points per axis (x, y, z), each >= 1 */
  double center;
  double lo[3];
  double hi[3];
  double shift_im;
} gadi_stencil;

/* Solver parameters.  Fill with gadi_params_default() first. */
typedef struct {
  double alpha;            /* regularization, > 0 (Section 2.1)                          */
  double omega;            /* extrapolation, in [0, 2) (Section 2.1)                      */
  int32_t u_r, u, u_s;     /* precisions; u = GADI_F64; u_r = GADI_F64 (default) or
                              GADI_F64X2 (fixed at gadi_create: it selects the kernels)  */
  int32_t stop_on_relres;  /* 0: backward error (default); 1: ||r||/||r0||                */
  double tol;              /* outer target, e.g. 1e-10                                    */
  int64_t max_outer;       /* sweep cap -> GADI_NOT_CONVERGED                             */
  int32_t stag_window;     /* outer stagnation window in sweeps (0: off), default 200     */
  int32_t inner_stag_window; /* inner early stop: no 1% progress in this many its (0: off) */
  double div_factor;       /* divergence if BE > div_factor * min BE (0: off), default 1e3 */
  double inner_tol_h;      /* relative-residual tolerance of CG on H (Section 5.1)        */
  double inner_tol_s;      /* relative-residual tolerance of CGNE on S                     */
  int32_t max_inner_h;     /* iteration caps of the inner solves                          */
  int32_t max_inner_s;
  int32_t fixed_inner_h;   /* > 0: run exactly this many CG iterations (mirror tests)     */
  int32_t fixed_inner_s;
  double normA;            /* > 0: use this ||A||_2; 0: estimate at gadi_create           */
  int32_t norm_iters;      /* power iterations for the estimate (default 100)             */
  int32_t tile_ry;         /* 3D tile rows per wave (1, 2 or 4); 0 (with tile_chunk 0): the
                              shape gadi_autotune chose for this class, else the library
                              default: 4 for FP64 / FP32 inner solves from 2^24 unknowns,
                              2 for BF16 from 2^26, 1 below those sizes and for complex */
  int32_t tile_chunk;      /* planes per tile along the marching axis of the inner tiling;
                              0: as tile_ry (the library default is the length that fills
                              the device in one round; 2D BF16 takes twice that while half
                              the resident waves still get a tile); -k (k in 1..64): both
                              tilings' chunks k times the one-round length, or the inner
                              one k times the tuned chunk of the class (k times fewer
                              tiles, for systems that share the device in a batch)       */
  int32_t max_restarts;    /* alpha restarts on outer stagnation or divergence (Section
                              4.3, step 3); 0 (default): none                            */
  double safeguard_tau;    /* > 0: before the solve, raise alpha until
                              kappa(H) kappa(S) u_s < safeguard_tau (the safety condition
                              of Section 4.3, step 2); 0 (default): no check.  Must exceed the unit
                              roundoff of u_s (Table 1).                                  */
  double alpha_growth;     /* factor of each alpha increase, > 1; default 10^(3/7), one
                              step of eight log-spaced values per decade triple          */
} gadi_params;

/* Outcome of a solve. */
typedef struct {
  int64_t outer;        /* sweeps performed (x returned is x^(outer))                */
  int64_t inner_h;      /* total CG iterations on H                                  */
  int64_t inner_s;      /* total CGNE iterations on S (0 for complex problems)       */
  double be;            /* backward error of the returned x (FP64, as computed)      */
  double relres;        /* ||r|| / ||r0||                                             */
  double normA;         /* ||A||_2 used in the backward error                        */
  double normb;
  double ms;            /* device time of the solve (hipEvent), milliseconds         */
  double kernel_ms;     /* hipEvent time of the step launches alone, i.e. the solve
                           without the host polls between launch chunks              */
  int32_t status;       /* GADI_OK .. GADI_DIVERGED                                   */
  int32_t steps;        /* device steps launched (including idle steps at the end)   */
  double alpha;         /* alpha of the last attempt (after the safeguard / restarts) */
  int32_t restarts;     /* alpha restarts performed                                  */
  int32_t attempt_outer; /* sweeps of the last attempt: h_history holds
                            attempt_outer + 1 entries (outer + 1 without restarts)    */
} gadi_report;

typedef struct gadi_handle gadi_handle;
typedef struct gadi_batch gadi_batch;

/* Library version string. */
const char* gadi_version(void);
/* Text of a status code. */
const char* gadi_status_string(gadi_status s);
/* Message of the last error on the calling thread ("" if none). */
const char* gadi_last_error(void);

/* Default parameters: alpha 0.5, omega 1, u_r = u = F64, u_s = F64, BE stop,
 * tol 1e-10, max_outer 20000, stag_window 200, inner_stag_window 20,
 * div_factor 1e3, inner tolerances 1e-3, caps 2000, normA estimated, no alpha
 * safeguard or restarts (alpha_growth 10^(3/7)). */
void gadi_params_default(gadi_params* p);

/* Bytes of device workspace a handle needs for (stencil, params); 256-byte
 * alignment is required.  Returns GADI_ERR_INVALID_ARG / UNSUPPORTED for
 * invalid or unsupported problems. */
gadi_status gadi_workspace_bytes(const gadi_stencil* st, const gadi_params* p, size_t* bytes);

/* Create a solver handle.  Validates arguments, lays out the workspace
 * (which must stay alive until gadi_destroy), zero-fills it, uploads the
 * operator description and, when p->normA == 0, estimates ||A||_2 by power
 * iteration on A^T A (a lower bound, so the backward error is conservative).
 * Synchronizes the stream before returning. */
gadi_status gadi_create(const gadi_stencil* st, const gadi_params* p, void* hip_stream,
                        void* d_workspace, size_t ws_bytes, gadi_handle** out);

/* Condition numbers of the two shifted splitting matrices for this stencil
 * and alpha (host only, closed forms of the constant-coefficient stencils,
 * Section 5 and the HSS splitting of Section 2.1):
 *   kappa(H) = (alpha + lambda_max(M)) / (alpha + lambda_min(M)),
 *   kappa(S) = sqrt(alpha^2 + rho(N)^2) / alpha  (an upper bound; exact when N
 *              has a zero eigenvalue),
 * with lambda(M) and rho(N) from the per-axis Toeplitz eigenvalues
 * c/dim + 2 m_d cos(j pi/(n_d+1)), m_d = (lo_d+hi_d)/2, and
 * i(shift_im + sum_d (hi_d-lo_d) cos(j_d pi/(n_d+1))).  Returns
 * GADI_ERR_INVALID_ARG for a null pointer, an invalid stencil or alpha <= 0,
 * and GADI_ERR_UNSUPPORTED when H is not positive definite for this alpha. */
gadi_status gadi_condition_estimate(const gadi_stencil* st, double alpha, double* kappa_H, double* kappa_S);

/* Change alpha / omega / tolerances of an existing handle (same operator and
 * precisions).  Must not be called while a solve is running. */
gadi_status gadi_set_params(gadi_handle* h, const gadi_params* p);

/* Solve A x = b.  d_b: device b (n values); d_x: device x, in: x^(0) (zeros
 * reproduce Algorithm 1), out: the returned iterate.  out may be NULL.
 * h_history (nullable, host, length 4*(max_outer+1)) receives per sweep k:
 * [BE_k, relres_k, CG iterations of sweep k, CGNE iterations of sweep k].
 * Blocks until the solve is finished.
 *
 * Alpha selection (Section 4.3): with safeguard_tau > 0 the solve starts from
 * the smallest alpha * alpha_growth^m (m >= 0) with kappa(H) kappa(S) u_s <
 * safeguard_tau (gadi_condition_estimate).  With max_restarts > 0, an attempt
 * that ends STAGNATED or DIVERGED is followed by another with alpha multiplied
 * by alpha_growth, starting from the last iterate after stagnation and from
 * zero after divergence; all attempts share the max_outer budget.  The report
 * sums sweeps and iterations over the attempts; h_history holds the last
 * attempt. */
gadi_status gadi_solve(gadi_handle* h, const void* d_b, void* d_x, gadi_report* out,
                       double* h_history);

/* Start a solve without waiting (same arguments as gadi_solve); progress it
 * with gadi_query.  b and x must stay alive until the solve has finished. */
gadi_status gadi_solve_async(gadi_handle* h, const void* d_b, void* d_x);

/* Advance / poll an asynchronous solve.  wait = 0: enqueue more device
 * steps if needed and return GADI_RUNNING while unfinished; wait = 1: run
 * to completion.  When finished, fills *out (nullable) and h_history. */
gadi_status gadi_query(gadi_handle* h, int32_t wait, gadi_report* out, double* h_history);

/* ||A||_2 in use by the handle (given or estimated). */
gadi_status gadi_get_norm(gadi_handle* h, double* normA);

/* Tile shape the handle's step kernel runs with (host only, no device work):
 * out[0] rows per wave of 3D tiles (1 in 2D), out[1] planes per chunk of the
 * inner (u_s) tiling, out[2] planes per chunk of the FP64 tiling, out[3]
 * blocks (tiles of four waves) of the larger tiling. */
gadi_status gadi_get_tiling(gadi_handle* h, int32_t out[4]);

/* Frees host state only; the caller frees the workspace afterwards. */
gadi_status gadi_destroy(gadi_handle* h);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1) in float64 / complex128
 * on dense vectors (the operator of Section 5, e.g. to form b = A x_true).
 * Asynchronous on the stream.  x and y must not overlap. */
gadi_status gadi_apply(const gadi_stencil* st, void* hip_stream, const void* d_x, void* d_y,
                       int32_t transpose);

/* r = b - A x on dense vectors: the residual step of Algorithm 1 (Section
 * 2.3) in precision u_r = GADI_F64 (plain FP64 arithmetic) or GADI_F64X2 (the
 * extra-precision arithmetic described at gadi_prec, identical to the
 * solver's residual with params.u_r = GADI_F64X2).  b, x, r: float64
 * (complex128 interleaved if st->is_complex) with n[0]*n[1]*n[2] elements,
 * x-fastest, caller-owned device memory.  r must not overlap b or x.
 * Asynchronous on the stream; GADI_ERR_INVALID_ARG for null pointers, an
 * invalid grid, an unknown u_r or overlapping r. */
gadi_status gadi_residual(const gadi_stencil* st, void* hip_stream, const void* d_b, const void* d_x, void* d_r,
                          int32_t u_r);

/* ---- data-driven initial alpha (Section 4.2) -------------------------------
 * Section 4.3 starts the alpha selection from a regression model trained on
 * small problems.  Features of a problem (closed forms of the stencil, host
 * only, no device work):
 *   f[0] = log10 lambda_min(M), f[1] = log10 lambda_max(M)      M = (A + A^H)/2
 *   f[2] = log10 max(rho(N), 1e-12)                               N = (A - A^H)/2
 *   f[3] = log10 of the unit roundoff of u_s (Table 1)
 * (per-axis Toeplitz eigenvalues summed over the axes; rho(N) adds |shift_im|
 * for complex problems).  GADI_ERR_UNSUPPORTED if M is not positive
 * definite, GADI_ERR_INVALID_ARG for an invalid grid or u_s. */
gadi_status gadi_alpha_features(const gadi_stencil* st, int32_t u_s, double f[4]);

/* Gaussian-process regression of log10(alpha_opt) on the features: linear
 * mean [1, f0, f1, f2, f3]^T b with b estimated from the data (flat prior),
 * squared-exponential covariance sf^2 exp(-1/2 sum_i ((f_i - f'_i)/l_i)^2)
 * and noise variance sn^2 (Rasmussen and Williams 2006, Section 2.7).
 * X: n_train x 4 features (row-major, host), y: n_train targets log10(alpha),
 * hyper = {l_0, l_1, l_2, l_3, sf, sn}, all > 0; n_train in [6, 4096].  The
 * model copies its inputs and factors them once (O(n_train^3) host work).
 * GADI_ERR_INVALID_ARG for bad sizes, non-finite or non-positive inputs, or a
 * covariance / basis matrix that is not positive definite. */
typedef struct gadi_alpha_gpr gadi_alpha_gpr;
gadi_status gadi_alpha_gpr_create(int32_t n_train, const double* X, const double* y, const double hyper[6],
                                  gadi_alpha_gpr** out);
/* Posterior mean of log10(alpha_opt) at features f, and (sd nullable) the
 * posterior standard deviation of the latent function, basis uncertainty
 * included. */
gadi_status gadi_alpha_gpr_predict(const gadi_alpha_gpr* m, const double f[4], double* log10_alpha, double* sd);
gadi_status gadi_alpha_gpr_destroy(gadi_alpha_gpr* m);

/* ---- batched execution ------------------------------------------------------
 * A batch advances many handles together: one device step launch per
 * (precision, dimension, tile shape) class moves every member by one phase
 * of its own state machine.  Steps are captured once in a hipGraph and
 * relaunched.  Results of a member do not depend on the other members
 * (each system keeps its own reduction order).  Members keep their Krylov
 * state resident in their own workspaces.  A member shares every launch
 * with the others, and each of its tiles pays a reduction and a ticket:
 * members created with tile_chunk = -k (k times fewer, longer tiles; k = 4
 * for the serving loop) make the batch's launches shorter.  The steps of
 * different kernel classes are captured as parallel graph branches. */

/* Device workspace of a batch able to hold max_systems members. */
gadi_status gadi_batch_workspace_bytes(int32_t max_systems, size_t* bytes);

gadi_status gadi_batch_create(int32_t max_systems, void* hip_stream, void* d_workspace,
                              size_t ws_bytes, gadi_batch** out);

/* Add a handle with its b and x (x^(0) in, result out); starts its solve.
 * The handle must use the batch's stream and must not be solving elsewhere.
 * *slot receives the member's slot id. */
gadi_status gadi_batch_add(gadi_batch* b, gadi_handle* h, const void* d_b, void* d_x,
                           int32_t* slot);

/* Launch nsteps device steps for all members (asynchronous). */
gadi_status gadi_batch_step(gadi_batch* b, int32_t nsteps);

/* Synchronize and report which members are finished: done[i] = 1 for slot i
 * if finished (length max_systems, nullable).  Returns the number of active
 * (unfinished) members through *active.  One small kernel gathers every
 * member's control block and one copy brings them to the host, after the
 * work already enqueued on the batch's stream. */
gadi_status gadi_batch_poll(gadi_batch* b, int32_t* done, int32_t* active);

/* Report of a finished member, then remove it from the batch. */
gadi_status gadi_batch_remove(gadi_batch* b, int32_t slot, gadi_report* out, double* h_history);

gadi_status gadi_batch_destroy(gadi_batch* b);

/* ---- autotuning -----------------------------------------------------------
 * Choose the tile shape of the step kernels (rows per wave in 3D: 1, 2 or 4;
 * planes per chunk of the inner tiling: half, once or twice the library's
 * default length) for this stencil's kernel class (dimension,
 * real / complex, u_s, u_r) and size class (floor(log2 n)) by timing each
 * candidate on the device: a handle is created in the caller's workspace
 * (ws_bytes must cover the largest candidate layout; gadi_workspace_bytes with
 * tile_ry = 1 and tile_chunk = 2 is an upper bound), the state machine is armed
 * with d_b / d_x (read only; x is not written) and whole sweeps (every phase:
 * the outer update and residual, 8 CG and 2 CGNE iterations) are timed with
 * hipEvents.  Returns the fastest shape for this grid in *ry, *chunk and its
 * time per sweep in *best_us.  The choice is kept for the class for the
 * process and, when the environment variable GADI_TUNE_CACHE names a file,
 * appended to it and read back by later processes; a class that already has
 * a choice is not timed again (*best_us = -1).  Every handle created
 * afterwards with tile_ry = tile_chunk = 0 (gadi_create, batches, the
 * allocation-free solve) runs with the shape chosen for its class, and one
 * with tile_ry = 0 and tile_chunk = -k with its rows per wave and k times its
 * chunk; create workspaces after tuning, since the shape changes the layout. */
gadi_status gadi_autotune(const gadi_stencil* st, const gadi_params* p, void* hip_stream,
                          void* d_workspace, size_t ws_bytes, const void* d_b, void* d_x,
                          int32_t* ry, int32_t* chunk, double* best_us);

/* ---- allocation-free solve -------------------------------------------------
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid it, set-ups that
 * record their other work into HIP graphs).  One whole solve, equivalent to
 * gadi_create + gadi_solve + gadi_destroy with the same stencil and
 * parameters (same kernels, same tile shape, same results), whose workspace
 * is a static device array of GADI_NOALLOC_SCRATCH_BYTES bytes inside the
 * library (one per GPU, created when the library's code is loaded on that GPU
 * and held until the process ends) instead of caller memory.  The call makes
 * no hipMalloc / hipFree, no pinned host allocation and no event.  The caller
 * passes b and x (x^(0) in, result out) as for gadi_solve, on the current
 * device.  A problem whose workspace (gadi_workspace_bytes) exceeds the limit
 * returns GADI_ERR_CAPACITY before any device work; with the default tile
 * shapes 64 MiB holds about 1.6e6 real unknowns with FP32 inner solves, 2.0e6
 * with BF16 and 1.1e6 with FP64.  All calls on one GPU share its array and
 * each call clears the part it uses before solving: calls that overlap on
 * one GPU (two threads, or two streams without ordering) race and corrupt
 * each other, so the caller serializes them.  The call synchronizes the
 * stream between launch chunks, so it cannot itself be captured in a graph.
 * The report's ms and kernel_ms are host-clock times of the call. */
#define GADI_NOALLOC_SCRATCH_BYTES (64u << 20)
gadi_status gadi_solve_noalloc(const gadi_stencil* st, const gadi_params* p, void* hip_stream,
                               const void* d_b, void* d_x, gadi_report* out, double* h_history);

#ifdef __cplusplus
}
#endif

#endif /* GADI_H */
