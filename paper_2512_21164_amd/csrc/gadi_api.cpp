// Host runtime and C ABI of the GADI library (declared in include/gadi.h).
//
// A handle owns no device memory: its workspace is carved into the system
// descriptor, the control block of the device state machine, reduction
// partials, the sweep history and the vectors.  A solve arms the state
// machine (IMPORT) and then launches device steps in chunks, reading the
// control block back between chunks until the machine reports DONE.  All
// decisions of Algorithm 1 (convergence, inner stopping, CG scalars) are
// taken on the device, so the host never waits on a dot product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gadi.h"
#include "gadi_internal.h"
#include "gadi_launch.h"

using namespace gadi;

namespace gadi {
// Copy the control block of each slot (src[i], null: none) to dst[i] (gadi_batch.hip).
hipError_t launch_gather_ctl(const GadiCtl* const* src, GadiCtl* dst, int n, hipStream_t st);
}  // namespace gadi

namespace {

thread_local std::string g_last_error;

gadi_status fail(gadi_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(GADI_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
constexpr int64_t kHistCap = 1 << 20;

struct Layout {
  int dim, cplx, us;
  int xr;                // residual with Dot2 sums (u_r = GADI_F64X2)
  int nx, ny, nz;
  int64_t P, nvec, n;
  int ny_plane, nm, RY, L, Lo, nwy;
  int64_t sy, sm;
  Tiling ti, to;
  int max_tiles;
  int64_t hist_len;
  size_t welem, selem;   // bytes of an FP64 element and of a u_s element
  // offsets
  size_t o_desc, o_ctl, o_counter, o_table, o_partials, o_hist, o_x0, o_x1, o_b, o_vs[4], total;
};

int us_bytes(int us, int cplx) {
  int b = us == US_F64 ? 8 : (us == US_F32 ? 4 : 2);
  return cplx ? 2 * b : b;
}

Tiling make_tiling(const Layout& l, int V, int L) {
  Tiling t{};
  t.V = V;
  t.L = L;
  t.nmc = (l.nm + L - 1) / L;
  t.nwx = (int)((l.nx + 64 * V - 1) / (64 * V));
  int64_t nwave = (int64_t)t.nwx * l.nwy * t.nmc;
  t.nwave = (int)nwave;
  t.ntiles = (int)((nwave + 3) / 4);
  return t;
}

gadi_status validate_stencil(const gadi_stencil* st) {
  if (!st) return fail(GADI_ERR_INVALID_ARG, "null stencil");
  if (st->dim != 2 && st->dim != 3) return fail(GADI_ERR_INVALID_ARG, "dim must be 2 or 3");
  for (int d = 0; d < 3; ++d)
    if (st->n[d] < 1) return fail(GADI_ERR_INVALID_ARG, "grid sizes must be >= 1");
  if (st->dim == 2 && st->n[2] != 1) return fail(GADI_ERR_INVALID_ARG, "2D problems need n[2] == 1");
  if (st->n[0] > (1 << 24) || st->n[1] > (1 << 24) || st->n[2] > (1 << 24))
    return fail(GADI_ERR_UNSUPPORTED, "grid side above 2^24");
  const double nn = (double)st->n[0] * (double)st->n[1] * (double)st->n[2];
  if (nn > 4.0e9) return fail(GADI_ERR_UNSUPPORTED, "more than 4e9 unknowns");
  if (!std::isfinite(st->center) || !std::isfinite(st->shift_im))
    return fail(GADI_ERR_INVALID_ARG, "non-finite stencil coefficient");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(st->lo[d]) || !std::isfinite(st->hi[d]))
      return fail(GADI_ERR_INVALID_ARG, "non-finite stencil coefficient");
  if (st->is_complex) {
    for (int d = 0; d < st->dim; ++d)
      if (st->lo[d] != st->hi[d])
        return fail(GADI_ERR_UNSUPPORTED, "complex problems need a symmetric real stencil (lo == hi)");
  } else if (st->shift_im != 0.0) {
    return fail(GADI_ERR_INVALID_ARG, "shift_im needs is_complex = 1");
  }
  return GADI_OK;
}

// Final statuses written by the device state machine (GADI_* values).
constexpr int ST_STAGNATED_H = GADI_STAGNATED;
constexpr int ST_DIVERGED_H = GADI_DIVERGED;

// Unit roundoff of a storage precision (Table 1).
double unit_roundoff(int us) {
  return us == GADI_F64 ? std::ldexp(1.0, -53) : (us == GADI_F32 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -8));
}

gadi_status validate(const gadi_stencil* st, const gadi_params* p) {
  if (!st || !p) return fail(GADI_ERR_INVALID_ARG, "null stencil or params");
  gadi_status vs = validate_stencil(st);
  if (vs != GADI_OK) return vs;
  if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(GADI_ERR_INVALID_ARG, "alpha must be > 0");
  if (!(p->omega >= 0.0 && p->omega < 2.0)) return fail(GADI_ERR_INVALID_ARG, "omega must lie in [0, 2)");
  if (p->u != GADI_F64) return fail(GADI_ERR_UNSUPPORTED, "u must be GADI_F64");
  if (p->u_r != GADI_F64 && p->u_r != GADI_F64X2)
    return fail(GADI_ERR_UNSUPPORTED, "u_r must be GADI_F64 or GADI_F64X2");
  if (p->u_s < GADI_F64 || p->u_s > GADI_BF16) return fail(GADI_ERR_INVALID_ARG, "unknown u_s");
  if (!(p->tol >= 0.0)) return fail(GADI_ERR_INVALID_ARG, "tol must be >= 0");
  if (p->max_outer < 0) return fail(GADI_ERR_INVALID_ARG, "max_outer must be >= 0");
  if (p->max_inner_h < 1 || p->max_inner_s < 1) return fail(GADI_ERR_INVALID_ARG, "inner caps must be >= 1");
  if (!(p->inner_tol_h >= 0.0) || !(p->inner_tol_s >= 0.0)) return fail(GADI_ERR_INVALID_ARG, "inner tolerances must be >= 0");
  if (p->fixed_inner_h < 0 || p->fixed_inner_s < 0 || p->stag_window < 0 || p->inner_stag_window < 0)
    return fail(GADI_ERR_INVALID_ARG, "negative iteration parameter");
  if (!(p->normA >= 0.0) || !std::isfinite(p->normA)) return fail(GADI_ERR_INVALID_ARG, "normA must be >= 0");
  if (p->normA == 0.0 && p->norm_iters < 1) return fail(GADI_ERR_INVALID_ARG, "norm_iters must be >= 1");
  if (p->tile_ry != 0 && p->tile_ry != 1 && p->tile_ry != 2 && p->tile_ry != 4)
    return fail(GADI_ERR_INVALID_ARG, "tile_ry must be 0, 1, 2 or 4");
  if (p->tile_chunk < -64 || p->tile_chunk > 4096) return fail(GADI_ERR_INVALID_ARG, "tile_chunk out of range");
  if (!(p->div_factor >= 0.0)) return fail(GADI_ERR_INVALID_ARG, "div_factor must be >= 0");
  if (p->max_restarts < 0 || p->max_restarts > 64) return fail(GADI_ERR_INVALID_ARG, "max_restarts must lie in [0, 64]");
  if (!(p->alpha_growth > 1.0) || !std::isfinite(p->alpha_growth))
    return fail(GADI_ERR_INVALID_ARG, "alpha_growth must be > 1");
  if (!(p->safeguard_tau >= 0.0) || !std::isfinite(p->safeguard_tau))
    return fail(GADI_ERR_INVALID_ARG, "safeguard_tau must be >= 0");
  if (p->safeguard_tau > 0.0 && !(p->safeguard_tau > unit_roundoff(p->u_s)))
    return fail(GADI_ERR_INVALID_ARG, "safeguard_tau must exceed the unit roundoff of u_s");
  return GADI_OK;
}

// Closed-form condition numbers of H = alpha I + M and S = alpha I + N for the
// constant-coefficient stencil (per-axis Toeplitz eigenvalues, Kronecker sums).
gadi_status condition_estimate(const gadi_stencil* st, double alpha, double* kH, double* kS) {
  const double pi = 3.14159265358979323846;
  double lmin = 0.0, lmax = 0.0, rho = std::fabs(st->shift_im);
  const double c = st->center / st->dim;
  for (int d = 0; d < st->dim; ++d) {
    const double cth = std::cos(pi / (double)(st->n[d] + 1));   // largest |cos(j pi/(n+1))|
    const double m = 0.5 * (st->lo[d] + st->hi[d]);
    const double nu = 0.5 * (st->hi[d] - st->lo[d]);
    lmin += c - 2.0 * std::fabs(m) * cth;
    lmax += c + 2.0 * std::fabs(m) * cth;
    rho += 2.0 * std::fabs(nu) * cth;
  }
  if (!(alpha + lmin > 0.0)) return fail(GADI_ERR_UNSUPPORTED, "alpha I + M is not positive definite");
  *kH = (alpha + lmax) / (alpha + lmin);
  *kS = std::sqrt(alpha * alpha + rho * rho) / alpha;
  return GADI_OK;
}

// Section 4.3, step 2: the smallest alpha * growth^m meeting kappa(H) kappa(S) u_s < tau.
gadi_status safeguarded_alpha(const gadi_stencil* st, const gadi_params& p, double* alpha) {
  double a = p.alpha;
  if (p.safeguard_tau > 0.0) {
    const double u = unit_roundoff(p.u_s);
    for (int it = 0;; ++it) {
      double kH = 0.0, kS = 0.0;
      gadi_status s = condition_estimate(st, a, &kH, &kS);
      if (s != GADI_OK) return s;
      if (kH * kS * u < p.safeguard_tau) break;
      if (it >= 4096 || !std::isfinite(a * p.alpha_growth))
        return fail(GADI_ERR_INVALID_ARG, "alpha safeguard cannot be met");
      a *= p.alpha_growth;
    }
  }
  *alpha = a;
  return GADI_OK;
}

// Waves of one kernel class resident on the whole device (with a fallback
// when no device is visible, e.g. for workspace sizing on a build host).
int64_t resident_waves(int us, int cplx, int dim, int ry, int xr) {
  static std::mutex mu;
  static std::map<int, int64_t> cache;
  const int key = (((us * 2 + cplx) * 4 + dim) * 8 + ry) * 2 + xr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0;
  int64_t waves = 256 * 4 * 4;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
    const int nb = step_blocks_per_cu(us, cplx, dim, ry, xr);
    if (nb > 0) waves = (int64_t)cus * nb * 4;
  } else {
    (void)hipGetLastError();
  }
  cache[key] = waves;
  return waves;
}

// Rows per wave of 3D tiles, by kernel class and grid size (fixed-iteration
// sweeps, microseconds per step launch over 32^3 .. 512^3).  Large grids are
// bandwidth bound and fewer halo rows pay: four rows for FP32 and FP64 from
// 2^24 unknowns (256^3: FP64 4% faster than one row, 512^3: FP32 9%), two
// for BF16 from 2^26 (512^3: 8%).  Below that a launch is short and bound by
// each wave's latency chain: one row per wave runs three waves per SIMD
// instead of one and is up to 38% faster (64^3 FP32: 8.7 against 14.1 us).
int default_ry(int us, int cplx, int64_t n) {
  if (cplx) return 1;
  if (us == US_BF16) return n >= (int64_t(1) << 26) ? 2 : 1;
  return n >= (int64_t(1) << 24) ? 4 : 1;
}

// Tile shapes chosen by the autotuner, per kernel class and size class:
// rows per wave and the inner chunk length as a multiple of the one-round
// default.  Handles created without an explicit tile shape use the entry of
// their class when there is one (see gadi_autotune).
struct TunedShape { int ry; double chunk_factor; };
std::mutex g_tune_mu;
std::map<std::string, TunedShape> g_tune_cache;
bool g_tune_file_read = false;

std::string tune_class_key(const gadi_stencil* st, const gadi_params* p) {
  const double n = (double)st->n[0] * (double)st->n[1] * (double)st->n[2];
  const int size_class = (int)std::floor(std::log2(std::max(1.0, n)));
  char buf[96];
  std::snprintf(buf, sizeof(buf), "d%d_c%d_u%d_x%d_n%d", st->dim, st->is_complex ? 1 : 0, p->u_s,
                p->u_r == GADI_F64X2 ? 1 : 0, size_class);
  return buf;
}

void load_tune_file_locked() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* f = std::getenv("GADI_TUNE_CACHE");
  if (!f) return;
  FILE* fp = std::fopen(f, "r");
  if (!fp) return;
  char key[96];
  int ry = 0;
  double fac = 0.0;
  while (std::fscanf(fp, "%95s %d %lf", key, &ry, &fac) == 3)
    if ((ry == 1 || ry == 2 || ry == 4) && fac > 0.0 && fac <= 64.0) g_tune_cache[key] = {ry, fac};
  std::fclose(fp);
}

bool tuned_shape(const gadi_stencil* st, const gadi_params* p, TunedShape* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tune_cache.find(tune_class_key(st, p));
  if (it == g_tune_cache.end()) return false;
  *out = it->second;
  return true;
}

// use_tuned: consult the autotuner's cache when p leaves the tile shape to the library
// (tile_ry 0 and tile_chunk 0, or tile_chunk -k: the tuned chunk k times longer)
Layout make_layout(const gadi_stencil* st, const gadi_params* p, bool use_tuned = true) {
  TunedShape tuned{0, 0.0};
  const bool have_tuned = use_tuned && p->tile_ry == 0 && p->tile_chunk <= 0 && tuned_shape(st, p, &tuned);
  Layout l{};
  l.dim = st->dim; l.cplx = st->is_complex ? 1 : 0; l.us = p->u_s;
  l.xr = p->u_r == GADI_F64X2 ? 1 : 0;
  l.nx = (int)st->n[0]; l.ny = (int)st->n[1]; l.nz = (int)st->n[2];
  l.P = (l.nx + 7) / 8 * 8;
  l.n = (int64_t)l.nx * l.ny * l.nz;
  l.nvec = l.P * l.ny * l.nz;
  if (l.dim == 2) {
    l.ny_plane = 1; l.nm = l.ny; l.sy = l.P; l.sm = l.P; l.RY = 1;
  } else {
    l.ny_plane = l.ny; l.nm = l.nz; l.sy = l.P; l.sm = l.P * l.ny;
    l.RY = p->tile_ry ? p->tile_ry : (have_tuned ? tuned.ry : default_ry(l.us, l.cplx, l.n));
  }
  l.nwy = (l.dim == 2) ? 1 : (l.ny_plane + l.RY - 1) / l.RY;
  // elements per lane of the inner phases (16-byte lane accesses)
  const int vi = l.cplx ? (l.us == US_F64 ? 1 : (l.us == US_F32 ? 2 : 4))
                        : (l.us == US_F64 ? 2 : (l.us == US_F32 ? 4 : GADI_BF16_V));
  // Chunk length of a tiling: one full round of resident waves (CUs x
  // resident blocks x 4 wave tiles), so that no launch ends with a partial
  // round.  tile_chunk > 0 overrides it for the inner tiling; tile_chunk = -k
  // makes both tilings' chunks k times longer (k times fewer tiles: for a
  // member of a batch, which shares the device with the other members).
  const int64_t waves = resident_waves(l.us, l.cplx, l.dim, l.RY, l.xr);
  auto one_round = [&](int V) -> int {
    const int64_t nwx = (l.nx + 64 * V - 1) / (64 * V);
    const int64_t per_plane = nwx * l.nwy;
    const int64_t chunks = std::max<int64_t>(1, waves / std::max<int64_t>(1, per_plane));
    const int64_t L = (l.nm + chunks - 1) / chunks;
    return (int)std::max<int64_t>(4, std::min<int64_t>(256, L));
  };
  const int vo = l.cplx ? 1 : 2;
  const int share = p->tile_chunk < 0 ? -p->tile_chunk : 1;
  auto scaled = [&](int L) -> int { return (int)std::min<int64_t>(std::max(l.nm, 1), (int64_t)L * share); };
  l.L = p->tile_chunk > 0 ? p->tile_chunk : scaled(one_round(vi));
  // 2D BF16 (real or pairs): with 16-byte lane accesses a one-round wave tile
  // is only a few rows long, and twice that is faster (4096^2: 26.6 -> 25.2
  // us per launch; complex 2048^2: 15.9 -> 15.4) as long as half the
  // resident waves still get a tile (small grids, whose one-round chunk is
  // already the minimum, lose: 1024^2 7.9 -> 9.2 us).
  if (p->tile_chunk == 0 && !have_tuned && l.dim == 2 && l.us == US_BF16) {
    const int L2 = 2 * l.L;
    const int64_t nwx = (l.nx + 64 * vi - 1) / (64 * vi);
    const int64_t tiles2 = nwx * ((l.nm + L2 - 1) / L2);
    if (2 * tiles2 >= waves) l.L = L2;
  }
  if (have_tuned) {
    const int64_t base = std::min<int64_t>(std::max(l.nm, 1), one_round(vi));
    const int64_t L1 = std::max<int64_t>(2, std::min<int64_t>(4096, std::llround(tuned.chunk_factor * base)));
    l.L = share == 1 ? (int)L1 : (int)std::min<int64_t>(std::max(l.nm, 1), L1 * share);
  }
  l.Lo = scaled(one_round(vo));
  l.ti = make_tiling(l, vi, l.L);
  l.to = make_tiling(l, vo, l.Lo);
  l.max_tiles = std::max(l.ti.ntiles, l.to.ntiles);
  l.hist_len = std::min<int64_t>(p->max_outer + 1, kHistCap);
  l.welem = l.cplx ? 16 : 8;
  l.selem = us_bytes(l.us, l.cplx);
  size_t o = 0;
  l.o_desc = o; o = align_up(o + sizeof(GadiDesc));
  l.o_ctl = o; o = align_up(o + sizeof(GadiCtl));
  l.o_counter = o; o = align_up(o + GADI_TICKET_BYTES);
  l.o_table = o; o = align_up(o + sizeof(BatchTable) + sizeof(GadiDesc*) + 2 * sizeof(int32_t) + 64);
  l.o_partials = o; o = align_up(o + 4 * sizeof(double) * (size_t)l.max_tiles);
  l.o_hist = o; o = align_up(o + 4 * sizeof(double) * (size_t)l.hist_len);
  // The stencil sweeps load whole 64-lane rows, so a wave at the end of the
  // last row reads up to one wave access (64 lanes x 16 bytes) past the
  // vector: every vector is followed by that much slack.
  const size_t tail = 64 * 16;
  l.o_x0 = o; o = align_up(o + l.welem * (size_t)l.nvec + tail);
  l.o_x1 = o; o = align_up(o + l.welem * (size_t)l.nvec + tail);
  l.o_b = o; o = align_up(o + l.welem * (size_t)l.nvec + tail);
  for (int i = 0; i < 4; ++i) { l.o_vs[i] = o; o = align_up(o + l.selem * (size_t)l.nvec + tail); }
  l.total = o;
  return l;
}

void fill_desc(GadiDesc& d, const Layout& l, const gadi_stencil* st, const gadi_params* p, char* ws) {
  std::memset(&d, 0, sizeof(d));
  d.dim = l.dim; d.cplx = l.cplx; d.us = l.us; d.RY = l.RY;
  d.nx = l.nx; d.ny = l.ny; d.nz = l.nz;
  d.P = l.P; d.n = l.n; d.nvec = l.nvec;
  d.ny_plane = l.ny_plane; d.nm = l.nm; d.nwy = l.nwy;
  d.sy = l.sy; d.sm = l.sm;
  d.ti = l.ti; d.to = l.to; d.max_tiles = l.max_tiles;
  // kernel axis order: 0 = x, 1 = in-plane y (3D), 2 = marching axis (2D: y, 3D: z)
  const int map2[3] = {0, -1, 1}, map3[3] = {0, 1, 2};
  const int* mp = l.dim == 2 ? map2 : map3;
  d.cA = st->center;
  d.shift_im = l.cplx ? st->shift_im : 0.0;
  for (int a = 0; a < 3; ++a) {
    const int s = mp[a];
    const double lo = s >= 0 ? st->lo[s] : 0.0, hi = s >= 0 ? st->hi[s] : 0.0;
    d.loA[a] = lo; d.hiA[a] = hi;
    d.mH[a] = 0.5 * (lo + hi);           // M = (A + A^T)/2
    d.nuS[a] = 0.5 * (hi - lo);          // N = (A - A^T)/2: N(i, i+e) = (hi - lo)/2
  }
  d.alpha = p->alpha;
  d.cH = p->alpha + st->center;
  d.gamma = (2.0 - p->omega) * p->alpha;
  if (l.cplx) {
    const double den = p->alpha * p->alpha + st->shift_im * st->shift_im;
    d.g_re = d.gamma * p->alpha / den;
    d.g_im = -d.gamma * st->shift_im / den;
  }
  d.cAf = (float)d.cA; d.shift_imf = (float)d.shift_im;
  for (int a = 0; a < 3; ++a) {
    d.loAf[a] = (float)d.loA[a]; d.hiAf[a] = (float)d.hiA[a];
    d.mHf[a] = (float)d.mH[a]; d.nuSf[a] = (float)d.nuS[a];
  }
  d.cHf = (float)d.cH; d.alphaf = (float)d.alpha; d.gammaf = (float)d.gamma;
  d.tol = p->tol; d.div_factor = p->div_factor;
  d.inner_tol_h = p->inner_tol_h; d.inner_tol_s = p->inner_tol_s;
  d.max_outer = p->max_outer;
  d.stop_relres = p->stop_on_relres ? 1 : 0;
  d.stag_window = p->stag_window; d.inner_stag = p->inner_stag_window;
  d.max_inner_h = p->max_inner_h; d.max_inner_s = p->max_inner_s;
  d.fixed_h = p->fixed_inner_h; d.fixed_s = p->fixed_inner_s;
  d.hist_len = (int32_t)l.hist_len;
  d.xbuf[0] = reinterpret_cast<double*>(ws + l.o_x0);
  d.xbuf[1] = reinterpret_cast<double*>(ws + l.o_x1);
  d.bpad = reinterpret_cast<double*>(ws + l.o_b);
  for (int i = 0; i < 4; ++i) d.vs[i] = ws + l.o_vs[i];
  d.user_b = nullptr; d.user_x = nullptr;
  d.partials = reinterpret_cast<double*>(ws + l.o_partials);
  d.counter = reinterpret_cast<uint32_t*>(ws + l.o_counter);
  d.ctl = reinterpret_cast<GadiCtl*>(ws + l.o_ctl);
  d.hist = reinterpret_cast<double*>(ws + l.o_hist);
}

int kernel_class_key(const Layout& l) { return (((l.us * 2 + l.cplx) * 4 + l.dim) * 8 + l.RY) * 2 + l.xr; }

}  // namespace

struct gadi_handle {
  gadi_stencil st;
  gadi_params p;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  Layout lay;
  GadiDesc hdesc;
  GadiDesc* d_desc;
  GadiCtl* d_ctl;
  BatchTable* d_table;
  GadiCtl* h_ctl;        // pinned readback buffer
  double normA;
  hipEvent_t ev0, ev1;   // around the solve (null: timed on the host instead)
  hipEvent_t ec0, ec1;   // around each chunk of step launches (null: not timed)
  double kernel_ms;
  std::chrono::steady_clock::time_point t_start;   // host clock at the start of the solve
  double host_ms;        // host-timed solve (handles without events)
  // asynchronous solve
  int running;
  int chunk;
  int64_t steps;
  int64_t max_steps;
  int in_batch;
  // alpha selection of the running solve (Section 4.3)
  double alpha_cur;
  int restarts;
  int64_t acc_outer, acc_inner_h, acc_inner_s, acc_steps;
  double acc_kernel_ms;
  void* x_user;
  const void* b_user;
};

namespace {

gadi_status read_ctl(gadi_handle* h) {
  HIP_TRY(hipMemcpyAsync(h->h_ctl, h->d_ctl, sizeof(GadiCtl), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return GADI_OK;
}

gadi_status launch_steps(gadi_handle* h, int count) {
  const int grid = (h->lay.max_tiles + 7) / 8 * 8;
  for (int i = 0; i < count; ++i) {
    const StepArgs args{h->d_table, h->d_desc, h->d_ctl};
    hipError_t e = launch_step(h->lay.us, h->lay.cplx, h->lay.dim, h->lay.RY, h->lay.xr, args, grid, h->stream);
    if (e != hipSuccess) return fail(GADI_ERR_HIP, std::string("step launch: ") + hipGetErrorString(e));
  }
  h->steps += count;
  return GADI_OK;
}

// Upper bound on the device steps of one solve (the state machine always ends).
int64_t step_bound(const gadi_params& p, int cplx) {
  const int64_t ih = p.fixed_inner_h > 0 ? p.fixed_inner_h : p.max_inner_h;
  const int64_t is = cplx ? 0 : (p.fixed_inner_s > 0 ? p.fixed_inner_s : p.max_inner_s);
  const int64_t per = 2 * ih + 2 * is + 3;   // + OUTER, the z fold after an even CG count, slack
  return (p.max_outer + 1) * per + 16;
}

gadi_status run_to(gadi_handle* h, int target_phase, bool wait, int64_t bound) {
  for (;;) {
    if (h->ec0) HIP_TRY(hipEventRecord(h->ec0, h->stream));
    gadi_status s = launch_steps(h, h->chunk);
    if (s != GADI_OK) return s;
    if (h->ec1) HIP_TRY(hipEventRecord(h->ec1, h->stream));
    s = read_ctl(h);
    if (s != GADI_OK) return s;
    float cms = 0.f;
    if (h->ec0 && hipEventElapsedTime(&cms, h->ec0, h->ec1) == hipSuccess) h->kernel_ms += cms;
    if (h->h_ctl->phase == target_phase) return GADI_OK;
    if (h->steps > bound) return fail(GADI_ERR_STATE, "device state machine did not finish within its step bound");
    h->chunk = std::min(h->chunk * 2, 256);
    if (!wait) return GADI_RUNNING;
  }
}

void fill_report(gadi_handle* h, gadi_report* out) {
  if (!out) return;
  const GadiCtl& c = *h->h_ctl;
  out->outer = h->acc_outer + c.k;
  out->inner_h = h->acc_inner_h + c.inner_h_total;
  out->inner_s = h->acc_inner_s + c.inner_s_total;
  out->be = c.be;
  out->relres = c.relres;
  out->normA = c.normA;
  out->normb = c.normb;
  if (h->ev0) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev0, h->ev1) != hipSuccess) ms = -1.f;
    out->ms = ms;
    out->kernel_ms = h->kernel_ms;
  } else {
    out->ms = h->host_ms;
    out->kernel_ms = h->host_ms;
  }
  out->status = c.status;
  out->steps = (int32_t)std::min<int64_t>(h->acc_steps + h->steps, INT32_MAX);
  out->alpha = h->alpha_cur;
  out->restarts = h->restarts;
  out->attempt_outer = c.k;
}

gadi_status copy_history(gadi_handle* h, double* hist) {
  if (!hist) return GADI_OK;
  const int64_t n = std::min<int64_t>((int64_t)h->h_ctl->k + 1, h->lay.hist_len);
  HIP_TRY(hipMemcpy(hist, h->ws + h->lay.o_hist, (size_t)n * 4 * sizeof(double), hipMemcpyDeviceToHost));
  return GADI_OK;
}

// Arm one attempt of the solve: descriptor with this alpha and sweep budget,
// the caller's b / x, the state machine at IMPORT.
gadi_status arm_attempt(gadi_handle* h, double alpha, int64_t max_outer) {
  gadi_params q = h->p;
  q.alpha = alpha;
  q.max_outer = max_outer;
  fill_desc(h->hdesc, h->lay, &h->st, &q, h->ws);
  HIP_TRY(hipMemcpyAsync(h->d_desc, &h->hdesc, sizeof(GadiDesc), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(launch_set_io(h->d_desc, static_cast<const double*>(h->b_user), static_cast<double*>(h->x_user), h->stream));
  HIP_TRY(launch_set_phase(h->d_ctl, PH_IMPORT, 0, 0.0, h->stream));
  h->steps = 0;
  h->chunk = 16;
  h->max_steps = step_bound(q, h->lay.cplx);
  return GADI_OK;
}

gadi_status start_solve(gadi_handle* h, const void* b, void* x) {
  if (!b || !x) return fail(GADI_ERR_INVALID_ARG, "null b or x");
  if (h->running || h->in_batch) return fail(GADI_ERR_STATE, "a solve is already running on this handle");
  double alpha = h->p.alpha;
  gadi_status s = safeguarded_alpha(&h->st, h->p, &alpha);
  if (s != GADI_OK) return s;
  h->b_user = b;
  h->x_user = x;
  h->alpha_cur = alpha;
  h->restarts = 0;
  h->acc_outer = h->acc_inner_h = h->acc_inner_s = h->acc_steps = 0;
  h->kernel_ms = 0.0;
  h->t_start = std::chrono::steady_clock::now();
  if (h->ev0) HIP_TRY(hipEventRecord(h->ev0, h->stream));
  s = arm_attempt(h, alpha, h->p.max_outer);
  if (s != GADI_OK) return s;
  h->running = 1;
  return GADI_OK;
}

// Section 4.3, step 3: after an attempt that stagnated or diverged, stop,
// raise alpha and start again (from the last iterate after stagnation, from
// zero after divergence) while restarts and sweeps remain.
bool wants_restart(const gadi_handle* h) {
  const GadiCtl& c = *h->h_ctl;
  return (c.status == ST_STAGNATED_H || c.status == ST_DIVERGED_H) && h->restarts < h->p.max_restarts &&
         h->acc_outer + c.k < h->p.max_outer;
}

gadi_status restart_solve(gadi_handle* h) {
  const GadiCtl& c = *h->h_ctl;
  const bool diverged = c.status == ST_DIVERGED_H;
  h->acc_outer += c.k;
  h->acc_inner_h += c.inner_h_total;
  h->acc_inner_s += c.inner_s_total;
  h->acc_steps += h->steps;
  h->restarts += 1;
  h->alpha_cur *= h->p.alpha_growth;
  if (diverged) {
    const size_t elem = h->lay.cplx ? 16 : 8;
    HIP_TRY(hipMemsetAsync(h->x_user, 0, elem * (size_t)h->lay.n, h->stream));
  }
  gadi_status s = arm_attempt(h, h->alpha_cur, h->p.max_outer - h->acc_outer);
  if (s != GADI_OK) return s;
  h->h_ctl->phase = PH_IMPORT;   // host view until the next read of the control block
  return GADI_OK;
}

gadi_status finish_solve(gadi_handle* h, gadi_report* out, double* hist) {
  if (h->ev1) {
    HIP_TRY(hipEventRecord(h->ev1, h->stream));
    HIP_TRY(hipEventSynchronize(h->ev1));
  } else {
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  h->host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h->t_start).count();
  h->running = 0;
  fill_report(h, out);
  gadi_status s = copy_history(h, hist);
  if (s != GADI_OK) return s;
  return h->h_ctl->status;
}

// Lay a handle out over its workspace: descriptor, the single-system table,
// a zeroed workspace, and ||A||_2 (given, or estimated by power iteration).
// h->h_ctl must point at host memory for the control-block readback; the
// events are optional (null: no device timing).  zero_fill clears the
// workspace with a kernel on the stream (null: hipMemsetAsync).
gadi_status setup_handle(gadi_handle* h, const gadi_stencil* st, const gadi_params* p, hipStream_t stream, char* ws,
                         size_t ws_bytes, const Layout& l,
                         hipError_t (*zero_fill)(void*, size_t, hipStream_t)) {
  h->st = *st; h->p = *p;
  h->stream = stream;
  h->ws = ws;
  h->ws_bytes = ws_bytes;
  h->lay = l;
  h->d_desc = reinterpret_cast<GadiDesc*>(h->ws + l.o_desc);
  h->d_ctl = reinterpret_cast<GadiCtl*>(h->ws + l.o_ctl);
  h->d_table = reinterpret_cast<BatchTable*>(h->ws + l.o_table);
  fill_desc(h->hdesc, l, st, p, h->ws);
  // single-system table: desc pointer and tile prefix live right after the table header
  char* tb = h->ws + l.o_table;
  BatchTable t{};
  t.nsys = 1;
  t.total_tiles = l.max_tiles;
  t.slots = (l.max_tiles + 7) / 8 * 8;
  t.desc = reinterpret_cast<GadiDesc**>(tb + sizeof(BatchTable));
  t.tile_start = reinterpret_cast<int32_t*>(tb + sizeof(BatchTable) + sizeof(GadiDesc*));
  char tbuf[sizeof(BatchTable) + sizeof(GadiDesc*) + 2 * sizeof(int32_t)];
  std::memcpy(tbuf, &t, sizeof(t));
  std::memcpy(tbuf + sizeof(BatchTable), &h->d_desc, sizeof(GadiDesc*));
  int32_t ts[2] = {0, l.max_tiles};
  std::memcpy(tbuf + sizeof(BatchTable) + sizeof(GadiDesc*), ts, sizeof(ts));
  hipError_t e = zero_fill ? zero_fill(h->ws, l.total, h->stream) : hipMemsetAsync(h->ws, 0, l.total, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->d_desc, &h->hdesc, sizeof(GadiDesc), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(tb, tbuf, sizeof(tbuf), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(GADI_ERR_HIP, std::string("workspace init: ") + hipGetErrorString(e));
  if (p->normA > 0.0) {
    h->normA = p->normA;
    e = launch_set_norm(h->d_ctl, p->normA, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(GADI_ERR_HIP, std::string("set norm: ") + hipGetErrorString(e));
  } else {
    // power iteration on A^H A from a checkerboard start (2 steps per iteration)
    e = launch_set_phase(h->d_ctl, PH_NORM_A, p->norm_iters, 1.0 / std::sqrt((double)l.n), h->stream);
    if (e != hipSuccess) return fail(GADI_ERR_HIP, std::string("set phase: ") + hipGetErrorString(e));
    h->steps = 0;
    gadi_status s = launch_steps(h, 2 * p->norm_iters);
    if (s == GADI_OK) s = read_ctl(h);
    if (s != GADI_OK) return s;
    if (h->h_ctl->phase != PH_IDLE) return fail(GADI_ERR_STATE, "norm estimation did not finish");
    h->normA = h->h_ctl->normA;
  }
  return GADI_OK;
}

}  // namespace

extern "C" gadi_status gadi_solve(gadi_handle* h, const void* d_b, void* d_x, gadi_report* out, double* h_history);

namespace gadi {

// One whole solve (set-up, Algorithm 1, end) over device memory the caller
// provides, allocating nothing: the handle and the host copy of the control
// block live on this function's stack and no events are created (the report
// carries host-clock times).
int32_t solve_in_place(const gadi_stencil* st, const gadi_params* p, void* hip_stream, void* ws, size_t ws_cap,
                       hipError_t (*zero_fill)(void*, size_t, hipStream_t), const void* d_b, void* d_x,
                       gadi_report* out, double* h_history) {
  gadi_status s = validate(st, p);
  if (s != GADI_OK) return s;
  if (!d_b || !d_x) return fail(GADI_ERR_INVALID_ARG, "null b or x");
  if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(GADI_ERR_WORKSPACE, "bad scratch address");
  const Layout l = make_layout(st, p);
  if (l.total > ws_cap)
    return fail(GADI_ERR_CAPACITY, "problem needs " + std::to_string(l.total) + " bytes of device workspace; "
                                   "the allocation-free solve has " + std::to_string(ws_cap));
  gadi_handle h{};
  GadiCtl ctl{};
  h.h_ctl = &ctl;
  s = setup_handle(&h, st, p, static_cast<hipStream_t>(hip_stream), static_cast<char*>(ws), ws_cap, l, zero_fill);
  if (s != GADI_OK) return s;
  return gadi_solve(&h, d_b, d_x, out, h_history);
}

}  // namespace gadi

namespace {
}  // namespace

extern "C" {

const char* gadi_version(void) { return "gadi-mi355x 0.1 (gfx950)"; }

const char* gadi_status_string(gadi_status s) {
  switch (s) {
    case GADI_OK: return "OK";
    case GADI_NOT_CONVERGED: return "NOT_CONVERGED";
    case GADI_STAGNATED: return "STAGNATED";
    case GADI_DIVERGED: return "DIVERGED";
    case GADI_RUNNING: return "RUNNING";
    case GADI_ERR_INVALID_ARG: return "ERR_INVALID_ARG";
    case GADI_ERR_UNSUPPORTED: return "ERR_UNSUPPORTED";
    case GADI_ERR_WORKSPACE: return "ERR_WORKSPACE";
    case GADI_ERR_HIP: return "ERR_HIP";
    case GADI_ERR_CAPACITY: return "ERR_CAPACITY";
    case GADI_ERR_STATE: return "ERR_STATE";
    default: return "UNKNOWN";
  }
}

}  // extern "C"

int32_t gadi::set_error(int32_t status, const char* msg) { return fail(status, msg ? msg : ""); }

extern "C" {

const char* gadi_last_error(void) { return g_last_error.c_str(); }

void gadi_params_default(gadi_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->alpha = 0.5;
  p->omega = 1.0;
  p->u_r = GADI_F64; p->u = GADI_F64; p->u_s = GADI_F64;
  p->stop_on_relres = 0;
  p->tol = 1e-10;
  p->max_outer = 20000;
  p->stag_window = 200;
  p->inner_stag_window = 20;
  p->div_factor = 1e3;
  p->inner_tol_h = 1e-3;
  p->inner_tol_s = 1e-3;
  p->max_inner_h = 2000;
  p->max_inner_s = 2000;
  p->fixed_inner_h = 0;
  p->fixed_inner_s = 0;
  p->normA = 0.0;
  p->max_restarts = 0;
  p->safeguard_tau = 0.0;
  p->alpha_growth = std::pow(10.0, 3.0 / 7.0);
  p->norm_iters = 100;
  p->tile_ry = 0;
  p->tile_chunk = 0;
}

gadi_status gadi_workspace_bytes(const gadi_stencil* st, const gadi_params* p, size_t* bytes) {
  if (!bytes) return fail(GADI_ERR_INVALID_ARG, "null bytes");
  gadi_status s = validate(st, p);
  if (s != GADI_OK) return s;
  *bytes = make_layout(st, p).total;
  return GADI_OK;
}

gadi_status gadi_create(const gadi_stencil* st, const gadi_params* p, void* hip_stream, void* d_workspace,
                        size_t ws_bytes, gadi_handle** out) {
  if (!out) return fail(GADI_ERR_INVALID_ARG, "null out");
  *out = nullptr;
  gadi_status s = validate(st, p);
  if (s != GADI_OK) return s;
  Layout l = make_layout(st, p);
  if (!d_workspace) return fail(GADI_ERR_WORKSPACE, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) return fail(GADI_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < l.total)
    return fail(GADI_ERR_WORKSPACE, "workspace too small: need " + std::to_string(l.total) + " bytes");
  gadi_handle* h = new gadi_handle();
  auto cleanup = [&](gadi_status e) {
    if (h->h_ctl) (void)hipHostFree(h->h_ctl);
    for (hipEvent_t ev : {h->ev0, h->ev1, h->ec0, h->ec1})
      if (ev) (void)hipEventDestroy(ev);
    delete h;
    return e;
  };
  if (hipHostMalloc(reinterpret_cast<void**>(&h->h_ctl), sizeof(GadiCtl), hipHostMallocDefault) != hipSuccess) {
    h->h_ctl = nullptr;
    return cleanup(fail(GADI_ERR_HIP, "pinned host buffer"));
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
      hipEventCreate(&h->ec0) != hipSuccess || hipEventCreate(&h->ec1) != hipSuccess)
    return cleanup(fail(GADI_ERR_HIP, "event create"));
  s = setup_handle(h, st, p, static_cast<hipStream_t>(hip_stream), static_cast<char*>(d_workspace), ws_bytes, l,
                   nullptr);
  if (s != GADI_OK) return cleanup(s);
  *out = h;
  return GADI_OK;
}

gadi_status gadi_condition_estimate(const gadi_stencil* st, double alpha, double* kappa_H, double* kappa_S) {
  if (!kappa_H || !kappa_S) return fail(GADI_ERR_INVALID_ARG, "null output");
  gadi_status s = validate_stencil(st);
  if (s != GADI_OK) return s;
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(GADI_ERR_INVALID_ARG, "alpha must be > 0");
  return condition_estimate(st, alpha, kappa_H, kappa_S);
}

gadi_status gadi_set_params(gadi_handle* h, const gadi_params* p) {
  if (!h || !p) return fail(GADI_ERR_INVALID_ARG, "null handle or params");
  if (h->running || h->in_batch) return fail(GADI_ERR_STATE, "solve running");
  gadi_status s = validate(&h->st, p);
  if (s != GADI_OK) return s;
  if (p->u_s != h->p.u_s) return fail(GADI_ERR_INVALID_ARG, "u_s cannot change");
  if (p->u_r != h->p.u_r) return fail(GADI_ERR_INVALID_ARG, "u_r cannot change");
  Layout l = make_layout(&h->st, p);
  if (l.total > h->ws_bytes || l.max_tiles != h->lay.max_tiles || l.RY != h->lay.RY || l.L != h->lay.L ||
      l.Lo != h->lay.Lo)
    return fail(GADI_ERR_INVALID_ARG, "new parameters change the workspace layout; create a new handle");
  GadiDesc d;
  fill_desc(d, l, &h->st, p, h->ws);
  HIP_TRY(hipMemcpyAsync(h->d_desc, &d, sizeof(GadiDesc), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->hdesc = d;
  h->lay = l;
  const double keep = h->normA;
  h->p = *p;
  if (p->normA > 0.0) {
    h->normA = p->normA;
    HIP_TRY(launch_set_norm(h->d_ctl, p->normA, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  } else {
    h->normA = keep;
  }
  return GADI_OK;
}

gadi_status gadi_solve(gadi_handle* h, const void* d_b, void* d_x, gadi_report* out, double* h_history) {
  if (!h) return fail(GADI_ERR_INVALID_ARG, "null handle");
  gadi_status s = start_solve(h, d_b, d_x);
  if (s != GADI_OK) return s;
  for (;;) {
    s = run_to(h, PH_DONE, true, h->max_steps);
    if (s != GADI_OK) { h->running = 0; return s; }
    if (!wants_restart(h)) break;
    s = restart_solve(h);
    if (s != GADI_OK) { h->running = 0; return s; }
  }
  return finish_solve(h, out, h_history);
}

gadi_status gadi_solve_async(gadi_handle* h, const void* d_b, void* d_x) {
  if (!h) return fail(GADI_ERR_INVALID_ARG, "null handle");
  gadi_status s = start_solve(h, d_b, d_x);
  if (s != GADI_OK) return s;
  return launch_steps(h, h->chunk);
}

gadi_status gadi_query(gadi_handle* h, int32_t wait, gadi_report* out, double* h_history) {
  if (!h) return fail(GADI_ERR_INVALID_ARG, "null handle");
  if (!h->running) return fail(GADI_ERR_STATE, "no solve running");
  gadi_status s = read_ctl(h);
  if (s != GADI_OK) return s;
  for (;;) {
    if (h->h_ctl->phase != PH_DONE) {
      s = run_to(h, PH_DONE, wait != 0, h->max_steps);
      if (s == GADI_RUNNING) return s;
      if (s != GADI_OK) { h->running = 0; return s; }
    }
    if (!wants_restart(h)) break;
    s = restart_solve(h);
    if (s != GADI_OK) { h->running = 0; return s; }
  }
  return finish_solve(h, out, h_history);
}

gadi_status gadi_get_norm(gadi_handle* h, double* normA) {
  if (!h || !normA) return fail(GADI_ERR_INVALID_ARG, "null argument");
  *normA = h->normA;
  return GADI_OK;
}

gadi_status gadi_get_tiling(gadi_handle* h, int32_t out[4]) {
  if (!h || !out) return fail(GADI_ERR_INVALID_ARG, "null argument");
  out[0] = h->lay.RY;
  out[1] = h->lay.L;
  out[2] = h->lay.Lo;
  out[3] = h->lay.max_tiles;
  return GADI_OK;
}

gadi_status gadi_destroy(gadi_handle* h) {
  if (!h) return GADI_OK;
  (void)hipStreamSynchronize(h->stream);
  (void)hipEventDestroy(h->ev0);
  (void)hipEventDestroy(h->ev1);
  (void)hipEventDestroy(h->ec0);
  (void)hipEventDestroy(h->ec1);
  if (h->h_ctl) (void)hipHostFree(h->h_ctl);
  delete h;
  return GADI_OK;
}

}  // extern "C"

namespace {
// Grid checks of the dense utility entry points (one thread per unknown).
gadi_status check_dense_grid(const gadi_stencil* st) {
  if (st->dim != 2 && st->dim != 3) return fail(GADI_ERR_INVALID_ARG, "dim must be 2 or 3");
  for (int d = 0; d < 3; ++d)
    if (st->n[d] < 1 || st->n[d] > INT32_MAX) return fail(GADI_ERR_INVALID_ARG, "grid sizes must lie in [1, 2^31)");
  if (st->dim == 2 && st->n[2] != 1) return fail(GADI_ERR_INVALID_ARG, "2D problems need n[2] == 1");
  if (st->n[0] * st->n[1] > INT64_MAX / st->n[2]) return fail(GADI_ERR_INVALID_ARG, "grid too large");
  return GADI_OK;
}
}  // namespace

extern "C" {

gadi_status gadi_apply(const gadi_stencil* st, void* hip_stream, const void* d_x, void* d_y, int32_t transpose) {
  if (!st || !d_x || !d_y) return fail(GADI_ERR_INVALID_ARG, "null argument");
  gadi_status s = check_dense_grid(st);
  if (s != GADI_OK) return s;
  if (d_x == d_y) return fail(GADI_ERR_INVALID_ARG, "x and y must not overlap");
  double lo[3] = {st->lo[0], st->lo[1], st->dim == 3 ? st->lo[2] : 0.0};
  double hi[3] = {st->hi[0], st->hi[1], st->dim == 3 ? st->hi[2] : 0.0};
  HIP_TRY(launch_apply_dense(st->is_complex ? 1 : 0, st->dim, (int)st->n[0], (int)st->n[1], (int)st->n[2], st->center,
                             lo, hi, st->is_complex ? st->shift_im : 0.0, transpose ? 1 : 0,
                             static_cast<const double*>(d_x), static_cast<double*>(d_y),
                             static_cast<hipStream_t>(hip_stream)));
  return GADI_OK;
}

gadi_status gadi_residual(const gadi_stencil* st, void* hip_stream, const void* d_b, const void* d_x, void* d_r,
                          int32_t u_r) {
  if (!st || !d_b || !d_x || !d_r) return fail(GADI_ERR_INVALID_ARG, "null argument");
  gadi_status s = check_dense_grid(st);
  if (s != GADI_OK) return s;
  if (u_r != GADI_F64 && u_r != GADI_F64X2) return fail(GADI_ERR_INVALID_ARG, "u_r must be GADI_F64 or GADI_F64X2");
  if (d_r == d_b || d_r == d_x) return fail(GADI_ERR_INVALID_ARG, "r must not overlap b or x");
  HIP_TRY(launch_residual_dense(st->is_complex ? 1 : 0, u_r == GADI_F64X2 ? 1 : 0, st->dim, (int)st->n[0],
                                (int)st->n[1], (int)st->n[2], st->center, st->lo, st->hi,
                                st->is_complex ? st->shift_im : 0.0, static_cast<const double*>(d_b),
                                static_cast<const double*>(d_x), static_cast<double*>(d_r),
                                static_cast<hipStream_t>(hip_stream)));
  return GADI_OK;
}

}  // extern "C"

// ============================================================== batches
// A batch keeps one device table per kernel class (u_s, complex, dimension,
// rows per wave).  Each step launch of a class uses a persistent grid that
// walks the tiles of all members of the class, so membership changes only
// rewrite the tables; the captured hipGraph is rebuilt only when the set of
// classes, a class of one system (its pointers are kernel arguments) or the
// number of steps per launch changes.
namespace {

struct ClassGroup {
  int key;
  int us, cplx, dim, ry, xr;
  int nsys;
  BatchTable* d_table;        // device table header
  GadiDesc** d_desc;          // device array of descriptor pointers
  int32_t* d_start;           // device prefix sums
  const GadiDesc* one = nullptr;  // a group of one system: its descriptor
  const GadiCtl* one_ctl = nullptr;  // and control block (step kernel arguments)
};

}  // namespace

struct gadi_batch {
  int max_sys;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  std::vector<gadi_handle*> member;   // by slot (nullptr = free)
  std::vector<int> done;              // by slot
  std::vector<ClassGroup> groups;     // classes present, in key order
  std::vector<int> graph_keys;        // classes captured in the graph
  std::vector<const void*> graph_args;  // single-system kernel arguments captured in the graph
  bool dirty;
  hipGraph_t graph;
  hipGraphExec_t exec;
  int graph_steps;
  GadiCtl* h_ctls;                    // pinned readback of all members' control blocks
  GadiCtl** d_ctl_src;                // device: control block of each slot's member (null: none)
  GadiCtl* d_ctl_dst;                 // device: the gathered control blocks, one per slot
  // graph branches: class g > 0 is captured on side[g], forked from and joined back into stream
  hipStream_t side[8];
  hipEvent_t fork_ev;
  hipEvent_t join_ev[8];
  bool branches_ready;
};

namespace {

constexpr int kMaxGroups = 8;
static_assert(sizeof(gadi_batch::side) / sizeof(hipStream_t) == kMaxGroups, "one side stream per class");
constexpr int kGroupGrid = 2048;     // persistent grid of a batch step launch (multiple of 8)

size_t group_bytes(int max_sys) {
  return align_up(sizeof(BatchTable)) + align_up(sizeof(GadiDesc*) * (size_t)max_sys) +
         align_up(sizeof(int32_t) * (size_t)(max_sys + 1));
}

// Batch workspace: the class tables, then the slot -> control block pointers
// and the gathered control blocks of a poll.
size_t batch_bytes(int max_sys) {
  return kMaxGroups * group_bytes(max_sys) + align_up(sizeof(GadiCtl*) * (size_t)max_sys) +
         align_up(sizeof(GadiCtl) * (size_t)max_sys);
}

gadi_status rebuild_tables(gadi_batch* b) {
  std::map<int, std::vector<int>> by;
  for (int i = 0; i < b->max_sys; ++i)
    if (b->member[i] && !b->done[i]) by[kernel_class_key(b->member[i]->lay)].push_back(i);
  if ((int)by.size() > kMaxGroups) return fail(GADI_ERR_CAPACITY, "too many kernel classes in one batch");
  std::vector<ClassGroup> groups;
  int gi = 0;
  for (auto& kv : by) {
    ClassGroup g{};
    const Layout& l0 = b->member[kv.second[0]]->lay;
    g.key = kv.first;
    g.us = l0.us; g.cplx = l0.cplx; g.dim = l0.dim; g.ry = l0.RY; g.xr = l0.xr;
    g.nsys = (int)kv.second.size();
    char* base = b->ws + gi * group_bytes(b->max_sys);
    g.d_table = reinterpret_cast<BatchTable*>(base);
    g.d_desc = reinterpret_cast<GadiDesc**>(base + align_up(sizeof(BatchTable)));
    g.d_start = reinterpret_cast<int32_t*>(base + align_up(sizeof(BatchTable)) +
                                           align_up(sizeof(GadiDesc*) * (size_t)b->max_sys));
    std::vector<GadiDesc*> descs;
    std::vector<int32_t> start{0};
    for (int s : kv.second) {
      descs.push_back(b->member[s]->d_desc);
      start.push_back(start.back() + b->member[s]->lay.max_tiles);
    }
    BatchTable t{};
    t.nsys = g.nsys;
    t.total_tiles = start.back();
    t.slots = (t.total_tiles + 7) / 8 * 8;
    t.desc = g.d_desc;
    t.tile_start = g.d_start;
    if (g.nsys == 1) {
      g.one = b->member[kv.second[0]]->d_desc;
      g.one_ctl = b->member[kv.second[0]]->d_ctl;
    }
    HIP_TRY(hipMemcpyAsync(g.d_desc, descs.data(), descs.size() * sizeof(GadiDesc*), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(g.d_start, start.data(), start.size() * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(g.d_table, &t, sizeof(t), hipMemcpyHostToDevice, b->stream));
    // the host vectors are pageable: let the copies consume them before they go out of scope
    HIP_TRY(hipStreamSynchronize(b->stream));
    groups.push_back(g);
    ++gi;
  }
  std::vector<int> keys;
  std::vector<const void*> args;
  for (auto& g : groups) {
    keys.push_back(g.key);
    args.push_back(g.one);
    args.push_back(g.one_ctl);
  }
  // the graph holds the kernel arguments: rebuild it when they change too
  if (keys != b->graph_keys || args != b->graph_args) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  }
  // slot -> control block of an unfinished member, for the gather of a poll
  std::vector<GadiCtl*> src(b->max_sys, nullptr);
  for (int i = 0; i < b->max_sys; ++i)
    if (b->member[i] && !b->done[i]) src[i] = b->member[i]->d_ctl;
  HIP_TRY(hipMemcpyAsync(b->d_ctl_src, src.data(), src.size() * sizeof(GadiCtl*), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->groups = groups;
  b->dirty = false;
  return GADI_OK;
}

gadi_status launch_groups(gadi_batch* b, int nsteps) {
  for (int s = 0; s < nsteps; ++s)
    for (auto& g : b->groups) {
      hipError_t e = launch_step(g.us, g.cplx, g.dim, g.ry, g.xr, StepArgs{g.d_table, g.one, g.one_ctl}, kGroupGrid, b->stream);
      if (e != hipSuccess) return fail(GADI_ERR_HIP, std::string("batch step: ") + hipGetErrorString(e));
    }
  return GADI_OK;
}

// Side streams (default priority) and events for the graph branches, created on first use.
gadi_status ensure_branches(gadi_batch* b) {
  if (b->branches_ready) return GADI_OK;
  HIP_TRY(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
  for (int g = 1; g < kMaxGroups; ++g) {
    HIP_TRY(hipStreamCreateWithFlags(&b->side[g], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&b->join_ev[g], hipEventDisableTiming));
  }
  b->branches_ready = true;
  return GADI_OK;
}

// The launches of a captured batch step: the classes are independent (each
// member belongs to one class), so class 0 runs on the batch's stream and
// every other class on its own side stream, forked from the batch's stream
// and joined back into it.  The graph then holds one chain of nsteps
// launches per class, and chains of small members overlap on the device
// instead of running one after the other.
gadi_status launch_groups_branched(gadi_batch* b, int nsteps) {
  const int G = (int)b->groups.size();
  HIP_TRY(hipEventRecord(b->fork_ev, b->stream));
  for (int g = 1; g < G; ++g) HIP_TRY(hipStreamWaitEvent(b->side[g], b->fork_ev, 0));
  for (int s = 0; s < nsteps; ++s)
    for (int g = 0; g < G; ++g) {
      const ClassGroup& c = b->groups[g];
      hipError_t e = launch_step(c.us, c.cplx, c.dim, c.ry, c.xr, StepArgs{c.d_table, c.one, c.one_ctl}, kGroupGrid,
                                 g == 0 ? b->stream : b->side[g]);
      if (e != hipSuccess) return fail(GADI_ERR_HIP, std::string("batch step: ") + hipGetErrorString(e));
    }
  for (int g = 1; g < G; ++g) {
    HIP_TRY(hipEventRecord(b->join_ev[g], b->side[g]));
    HIP_TRY(hipStreamWaitEvent(b->stream, b->join_ev[g], 0));
  }
  return GADI_OK;
}

}  // namespace

extern "C" {

gadi_status gadi_batch_workspace_bytes(int32_t max_systems, size_t* bytes) {
  if (!bytes || max_systems < 1) return fail(GADI_ERR_INVALID_ARG, "bad arguments");
  *bytes = batch_bytes(max_systems);
  return GADI_OK;
}

gadi_status gadi_batch_create(int32_t max_systems, void* hip_stream, void* d_workspace, size_t ws_bytes,
                              gadi_batch** out) {
  if (!out || max_systems < 1) return fail(GADI_ERR_INVALID_ARG, "bad arguments");
  *out = nullptr;
  size_t need = batch_bytes(max_systems);
  if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % kAlign) return fail(GADI_ERR_WORKSPACE, "bad workspace");
  if (ws_bytes < need) return fail(GADI_ERR_WORKSPACE, "batch workspace too small");
  gadi_batch* b = new gadi_batch();
  b->max_sys = max_systems;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->ws = static_cast<char*>(d_workspace);
  b->ws_bytes = ws_bytes;
  b->member.assign(max_systems, nullptr);
  b->done.assign(max_systems, 0);
  b->dirty = true;
  b->graph = nullptr;
  b->exec = nullptr;
  b->graph_steps = 0;
  b->d_ctl_src = reinterpret_cast<GadiCtl**>(b->ws + kMaxGroups * group_bytes(max_systems));
  b->d_ctl_dst = reinterpret_cast<GadiCtl*>(b->ws + kMaxGroups * group_bytes(max_systems) +
                                            align_up(sizeof(GadiCtl*) * (size_t)max_systems));
  if (hipHostMalloc(reinterpret_cast<void**>(&b->h_ctls), sizeof(GadiCtl) * (size_t)max_systems,
                    hipHostMallocDefault) != hipSuccess) {
    delete b;
    return fail(GADI_ERR_HIP, "pinned host buffer");
  }
  *out = b;
  return GADI_OK;
}

gadi_status gadi_batch_add(gadi_batch* b, gadi_handle* h, const void* d_b, void* d_x, int32_t* slot) {
  if (!b || !h || !d_b || !d_x) return fail(GADI_ERR_INVALID_ARG, "null argument");
  if (h->running || h->in_batch) return fail(GADI_ERR_STATE, "handle busy");
  int free_slot = -1;
  for (int i = 0; i < b->max_sys; ++i)
    if (!b->member[i]) { free_slot = i; break; }
  if (free_slot < 0) return fail(GADI_ERR_CAPACITY, "batch full");
  // the handle was created (and synchronized) on its own stream; from now on
  // it is driven on the batch's stream
  h->stream = b->stream;
  gadi_status s = start_solve(h, d_b, d_x);
  if (s != GADI_OK) return s;
  h->running = 0;          // progress is driven by the batch
  h->in_batch = 1;
  b->member[free_slot] = h;
  b->done[free_slot] = 0;
  b->dirty = true;
  if (slot) *slot = free_slot;
  return GADI_OK;
}

gadi_status gadi_batch_step(gadi_batch* b, int32_t nsteps) {
  if (!b || nsteps < 0) return fail(GADI_ERR_INVALID_ARG, "bad arguments");
  if (b->dirty) {
    gadi_status s = rebuild_tables(b);
    if (s != GADI_OK) return s;
  }
  if (b->groups.empty() || nsteps == 0) return GADI_OK;
  if (b->stream == nullptr) {
    // the legacy default stream cannot be captured: launch directly
    gadi_status s = launch_groups(b, nsteps);
    if (s != GADI_OK) return s;
  } else {
    if (!b->exec || b->graph_steps != nsteps) {
      if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
      if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
      if (b->groups.size() > 1) {
        gadi_status sb = ensure_branches(b);
        if (sb != GADI_OK) return sb;
      }
      HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      gadi_status s = b->groups.size() > 1 ? launch_groups_branched(b, nsteps) : launch_groups(b, nsteps);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(b->stream, &g);
      if (s != GADI_OK) { if (g) (void)hipGraphDestroy(g); return s; }
      if (e != hipSuccess) return fail(GADI_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e));
      b->graph = g;
      HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->graph_steps = nsteps;
      b->graph_keys.clear();
      b->graph_args.clear();
      for (auto& gr : b->groups) {
        b->graph_keys.push_back(gr.key);
        b->graph_args.push_back(gr.one);
        b->graph_args.push_back(gr.one_ctl);
      }
    }
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  }
  for (int i = 0; i < b->max_sys; ++i)
    if (b->member[i] && !b->done[i]) b->member[i]->steps += nsteps;
  return GADI_OK;
}

gadi_status gadi_batch_poll(gadi_batch* b, int32_t* done, int32_t* active) {
  if (!b) return fail(GADI_ERR_INVALID_ARG, "null batch");
  if (b->dirty) {
    // membership changed since the last step: the gather must see the current members only
    gadi_status s = rebuild_tables(b);
    if (s != GADI_OK) return s;
  }
  // every member's control block in one gather kernel and one copy
  HIP_TRY(launch_gather_ctl(b->d_ctl_src, b->d_ctl_dst, b->max_sys, b->stream));
  HIP_TRY(hipMemcpyAsync(b->h_ctls, b->d_ctl_dst, sizeof(GadiCtl) * (size_t)b->max_sys, hipMemcpyDeviceToHost,
                         b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  int act = 0;
  bool changed = false;
  for (int i = 0; i < b->max_sys; ++i) {
    gadi_handle* h = b->member[i];
    if (!h) { if (done) done[i] = 0; continue; }
    if (!b->done[i] && b->h_ctls[i].phase == PH_DONE) {
      b->done[i] = 1;
      changed = true;
      *h->h_ctl = b->h_ctls[i];
      HIP_TRY(hipEventRecord(h->ev1, b->stream));
    }
    if (done) done[i] = b->done[i];
    if (!b->done[i]) ++act;
  }
  if (changed) b->dirty = true;
  if (active) *active = act;
  return GADI_OK;
}

gadi_status gadi_batch_remove(gadi_batch* b, int32_t slot, gadi_report* out, double* h_history) {
  if (!b || slot < 0 || slot >= b->max_sys || !b->member[slot]) return fail(GADI_ERR_INVALID_ARG, "bad slot");
  gadi_handle* h = b->member[slot];
  if (!b->done[slot]) return fail(GADI_ERR_STATE, "member not finished");
  HIP_TRY(hipEventSynchronize(h->ev1));
  fill_report(h, out);
  gadi_status s = copy_history(h, h_history);
  h->in_batch = 0;
  b->member[slot] = nullptr;
  b->done[slot] = 0;
  b->dirty = true;
  if (s != GADI_OK) return s;
  return h->h_ctl->status;
}

gadi_status gadi_batch_destroy(gadi_batch* b) {
  if (!b) return GADI_OK;
  (void)hipStreamSynchronize(b->stream);
  for (auto* h : b->member)
    if (h) h->in_batch = 0;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->h_ctls) (void)hipHostFree(b->h_ctls);
  if (b->branches_ready) {
    (void)hipEventDestroy(b->fork_ev);
    for (int g = 1; g < kMaxGroups; ++g) {
      (void)hipStreamDestroy(b->side[g]);
      (void)hipEventDestroy(b->join_ev[g]);
    }
  }
  delete b;
  return GADI_OK;
}

}  // extern "C"

// ============================================================== autotuning
namespace {

void save_tune_entry(const std::string& key, int ry, double factor) {
  const char* f = std::getenv("GADI_TUNE_CACHE");
  if (!f) return;
  FILE* fp = std::fopen(f, "a");
  if (!fp) return;
  std::fprintf(fp, "%s %d %.6g\n", key.c_str(), ry, factor);
  std::fclose(fp);
}

// Device steps of one sweep in the tuner's fixed-count solve: OUTER, then
// (H1 H2) per CG iteration, the z fold after an even CG count, then
// S0 S2 (S1 S2)^(CGNE iterations - 1).
constexpr int kTuneCG = 8, kTuneCGNE = 2;
int tune_steps_per_sweep(int us, int cplx, int dim, int ry) {
  return 1 + 2 * kTuneCG + (pairs_z(us, cplx, dim, ry) && kTuneCG % 2 == 0 ? 1 : 0) + (cplx ? 0 : 2 * kTuneCGNE);
}

// Time whole sweeps (every phase, 8 CG and 2 CGNE iterations each) with one
// tile shape; returns microseconds per sweep.
gadi_status time_shape(const gadi_stencil* st, const gadi_params* base, int ry, int L, hipStream_t stream, void* ws,
                       size_t ws_bytes, const void* b, void* x, double* us_per_sweep) {
  gadi_params q = *base;
  q.tile_ry = ry;
  q.tile_chunk = L;
  q.normA = 1.0;
  q.max_outer = 4;          // more than the sweeps run here: the machine stays in its sweeps
  q.fixed_inner_h = kTuneCG;
  q.fixed_inner_s = kTuneCGNE;
  q.tol = 0.0;
  q.stag_window = 0;
  q.div_factor = 0.0;
  q.max_restarts = 0;
  q.safeguard_tau = 0.0;
  size_t need = 0;
  gadi_status s = gadi_workspace_bytes(st, &q, &need);
  if (s != GADI_OK) return s;
  if (need > ws_bytes) return fail(GADI_ERR_WORKSPACE, "autotune workspace too small");
  gadi_handle* h = nullptr;
  s = gadi_create(st, &q, stream, ws, ws_bytes, &h);
  if (s != GADI_OK) return s;
  const int per = tune_steps_per_sweep(h->lay.us, h->lay.cplx, h->lay.dim, h->lay.RY), warm = 1, meas = 2;   // warm + meas < q.max_outer
  s = start_solve(h, b, x);
  if (s == GADI_OK) s = launch_steps(h, 1 + warm * per);           // IMPORT and a warm-up sweep
  hipEvent_t e0 = h->ec0, e1 = h->ec1;
  if (s == GADI_OK && hipEventRecord(e0, stream) != hipSuccess) s = fail(GADI_ERR_HIP, "event");
  if (s == GADI_OK) s = launch_steps(h, meas * per);
  if (s == GADI_OK && hipEventRecord(e1, stream) != hipSuccess) s = fail(GADI_ERR_HIP, "event");
  if (s == GADI_OK && hipEventSynchronize(e1) != hipSuccess) s = fail(GADI_ERR_HIP, "event sync");
  if (s == GADI_OK) s = read_ctl(h);
  if (s == GADI_OK && !(h->h_ctl->phase == PH_OUTER && h->h_ctl->k == warm + meas))
    s = fail(GADI_ERR_STATE, "autotune: the state machine is not at the start of a sweep after the timed steps");
  float ms = 0.f;
  if (s == GADI_OK) (void)hipEventElapsedTime(&ms, e0, e1);
  h->running = 0;
  gadi_destroy(h);
  if (s != GADI_OK) return s;
  *us_per_sweep = 1000.0 * ms / meas;
  return GADI_OK;
}

}  // namespace

extern "C" gadi_status gadi_autotune(const gadi_stencil* st, const gadi_params* p, void* hip_stream, void* d_workspace,
                                     size_t ws_bytes, const void* d_b, void* d_x, int32_t* ry, int32_t* chunk,
                                     double* best_us) {
  if (!ry || !chunk || !d_b || !d_x) return fail(GADI_ERR_INVALID_ARG, "null argument");
  gadi_status s = validate(st, p);
  if (s != GADI_OK) return s;
  const std::string key = tune_class_key(st, p);
  TunedShape known{0, 0.0};
  if (tuned_shape(st, p, &known)) {
    // this class is tuned already (in this process or in the GADI_TUNE_CACHE file)
    gadi_params q = *p;
    q.tile_ry = 0;
    q.tile_chunk = 0;
    const Layout l = make_layout(st, &q, true);
    *ry = l.RY;
    *chunk = l.L;
    if (best_us) *best_us = -1.0;
    return GADI_OK;
  }
  // candidates: every rows-per-wave value (3D) with the library's default chunk, its half and
  // its double; the choice is kept as a multiple of the one-round chunk (tile_chunk = -1),
  // which is what make_layout scales a tuned entry by
  const std::vector<int> rys = st->dim == 3 ? std::vector<int>{1, 2, 4} : std::vector<int>{1};
  const double factors[3] = {0.5, 1.0, 2.0};
  double best = 1e300, bfac = 1.0;
  int bry = 0, bL = 0;
  std::vector<std::pair<int, int>> seen;
  for (int r : rys) {
    gadi_params q = *p;
    q.tile_ry = r;
    q.tile_chunk = 0;
    const int Ldef = make_layout(st, &q, false).L;
    q.tile_chunk = -1;
    const int Lround = make_layout(st, &q, false).L;
    for (double f : factors) {
      const int L = (int)std::max<int64_t>(2, std::min<int64_t>(4096, std::llround(f * Ldef)));
      if (std::find(seen.begin(), seen.end(), std::make_pair(r, L)) != seen.end()) continue;
      seen.emplace_back(r, L);
      double us = 0.0;
      s = time_shape(st, p, r, L, static_cast<hipStream_t>(hip_stream), d_workspace, ws_bytes, d_b, d_x, &us);
      if (s != GADI_OK) return s;
      if (std::getenv("GADI_TUNE_VERBOSE"))
        std::fprintf(stderr, "gadi_autotune %s ry=%d chunk=%d: %.2f us per sweep\n", key.c_str(), r, L, us);
      if (us < best) { best = us; bry = r; bL = L; bfac = (double)L / (double)Lround; }
    }
  }
  *ry = bry;
  *chunk = bL;
  if (best_us) *best_us = best;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file_locked();
  g_tune_cache[key] = {bry, bfac};
  save_tune_entry(key, bry, bfac);
  return GADI_OK;
}
