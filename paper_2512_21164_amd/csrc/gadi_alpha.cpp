// Data-driven initial alpha (Section 4.2): problem features from closed forms
// of the stencil, and a Gaussian-process regression model of log10(alpha_opt)
// over them (declared in include/gadi.h).
//
// Model.  f in R^4 (gadi_alpha_features), latent g(f) = h(f)^T b + GP(0, k)
// with the linear basis h(f) = [1, f0, f1, f2, f3], squared-exponential
// covariance k(f, f') = sf^2 exp(-1/2 sum_i ((f_i - f'_i) / l_i)^2) and
// observation noise sn^2.  With a flat prior on b the posterior at f* is
//   b_hat = (H Ky^-1 H^T)^-1 H Ky^-1 y,          Ky = K + sn^2 I,
//   mean  = h*^T b_hat + k*^T Ky^-1 (y - H^T b_hat),
//   var   = k(f*, f*) - k*^T Ky^-1 k* + R^T (H Ky^-1 H^T)^-1 R,
//   R     = h* - H Ky^-1 k*,
// the standard result for explicit basis functions (Rasmussen and Williams,
// Gaussian Processes for Machine Learning, 2006, Section 2.7).  Everything is
// factored once at creation (Cholesky of Ky and of the 5 x 5 matrix); a
// prediction costs O(n_train) plus two triangular solves for the variance.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gadi.h"
#include "gadi_internal.h"

namespace {

constexpr int kF = 4;   // features
constexpr int kB = 5;   // basis functions
constexpr int kMaxTrain = 4096;

double unit_roundoff_of(int32_t us) {
  switch (us) {
    case GADI_F64: return std::ldexp(1.0, -53);
    case GADI_F32: return std::ldexp(1.0, -24);
    case GADI_BF16: return std::ldexp(1.0, -8);
    default: return 0.0;
  }
}

// In-place Cholesky A = L L^T of an n x n SPD matrix (row-major, lower part).
bool cholesky(std::vector<double>& a, int n) {
  for (int j = 0; j < n; ++j) {
    double d = a[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double l = std::sqrt(d);
    a[(size_t)j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double s = a[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
      a[(size_t)i * n + j] = s / l;
    }
  }
  return true;
}

// x <- L^-1 x, then (optionally) x <- L^-T x.
void forward(const std::vector<double>& L, int n, double* x) {
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
}
void backward(const std::vector<double>& L, int n, double* x) {
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
}

void basis(const double* f, double* h) {
  h[0] = 1.0;
  for (int i = 0; i < kF; ++i) h[1 + i] = f[i];
}

}  // namespace

struct gadi_alpha_gpr {
  int n;
  std::vector<double> X;        // n x kF
  double ell[kF], sf2, sn2;
  std::vector<double> L;        // Cholesky factor of Ky (n x n)
  std::vector<double> w;        // Ky^-1 (y - H^T b_hat)
  std::vector<double> G;        // Ky^-1 H^T, n x kB (column j contiguous: G[j * n + i])
  double b[kB];                 // b_hat
  std::vector<double> LA;       // Cholesky factor of H Ky^-1 H^T (kB x kB)

  double kern(const double* f, const double* g) const {
    double q = 0.0;
    for (int i = 0; i < kF; ++i) {
      const double t = (f[i] - g[i]) / ell[i];
      q += t * t;
    }
    return sf2 * std::exp(-0.5 * q);
  }
};

extern "C" {

gadi_status gadi_alpha_features(const gadi_stencil* st, int32_t u_s, double f[4]) {
  if (!st || !f) return gadi::set_error(GADI_ERR_INVALID_ARG, "null argument");
  if (st->dim != 2 && st->dim != 3) return gadi::set_error(GADI_ERR_INVALID_ARG, "dim must be 2 or 3");
  for (int d = 0; d < 3; ++d)
    if (st->n[d] < 1) return gadi::set_error(GADI_ERR_INVALID_ARG, "grid sizes must be >= 1");
  const double u = unit_roundoff_of(u_s);
  if (!(u > 0.0)) return gadi::set_error(GADI_ERR_INVALID_ARG, "unknown u_s");
  // per axis: M has the symmetric tridiagonal (m, c/dim, m), N the skew one (-nu, 0, nu);
  // their Toeplitz eigenvalues are c/dim + 2 m cos(j pi/(n+1)) and 2 i nu cos(j pi/(n+1)).
  const double pi = 3.14159265358979323846;
  const double c = st->center / st->dim;
  double lmin = 0.0, lmax = 0.0, rho = st->is_complex ? std::fabs(st->shift_im) : 0.0;
  for (int d = 0; d < st->dim; ++d) {
    const double cth = std::cos(pi / (double)(st->n[d] + 1));
    const double m = 0.5 * (st->lo[d] + st->hi[d]);
    const double nu = 0.5 * (st->hi[d] - st->lo[d]);
    lmin += c - 2.0 * std::fabs(m) * cth;
    lmax += c + 2.0 * std::fabs(m) * cth;
    rho += 2.0 * std::fabs(nu) * cth;
  }
  if (!(lmin > 0.0)) return gadi::set_error(GADI_ERR_UNSUPPORTED, "M is not positive definite");
  f[0] = std::log10(lmin);
  f[1] = std::log10(lmax);
  f[2] = std::log10(rho > 1e-12 ? rho : 1e-12);
  f[3] = std::log10(u);
  return GADI_OK;
}

gadi_status gadi_alpha_gpr_create(int32_t n_train, const double* X, const double* y, const double hyper[6],
                                  gadi_alpha_gpr** out) {
  if (!X || !y || !hyper || !out) return gadi::set_error(GADI_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (n_train <= kB || n_train > kMaxTrain)
    return gadi::set_error(GADI_ERR_INVALID_ARG, "n_train must lie in [6, 4096]");
  for (int i = 0; i < 6; ++i)
    if (!(hyper[i] > 0.0) || !std::isfinite(hyper[i]))
      return gadi::set_error(GADI_ERR_INVALID_ARG, "hyperparameters must be positive and finite");
  for (int64_t i = 0; i < (int64_t)n_train * kF; ++i)
    if (!std::isfinite(X[i])) return gadi::set_error(GADI_ERR_INVALID_ARG, "non-finite feature");
  for (int i = 0; i < n_train; ++i)
    if (!std::isfinite(y[i])) return gadi::set_error(GADI_ERR_INVALID_ARG, "non-finite target");
  gadi_alpha_gpr* m = new (std::nothrow) gadi_alpha_gpr();
  if (!m) return gadi::set_error(GADI_ERR_CAPACITY, "out of host memory");
  const int n = n_train;
  m->n = n;
  m->X.assign(X, X + (size_t)n * kF);
  for (int i = 0; i < kF; ++i) m->ell[i] = hyper[i];
  m->sf2 = hyper[4] * hyper[4];
  m->sn2 = hyper[5] * hyper[5];
  // Ky and its Cholesky factor
  m->L.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = m->kern(&m->X[(size_t)i * kF], &m->X[(size_t)j * kF]);
      if (i == j) v += m->sn2;
      m->L[(size_t)i * n + j] = v;
    }
  if (!cholesky(m->L, n)) {
    delete m;
    return gadi::set_error(GADI_ERR_INVALID_ARG, "covariance matrix is not positive definite");
  }
  // G = Ky^-1 H^T and v = Ky^-1 y
  m->G.assign((size_t)kB * n, 0.0);
  std::vector<double> v(y, y + n);
  forward(m->L, n, v.data());
  backward(m->L, n, v.data());
  for (int j = 0; j < kB; ++j) {
    double* g = &m->G[(size_t)j * n];
    for (int i = 0; i < n; ++i) {
      double h[kB];
      basis(&m->X[(size_t)i * kF], h);
      g[i] = h[j];
    }
    forward(m->L, n, g);
    backward(m->L, n, g);
  }
  // A = H Ky^-1 H^T (kB x kB), rhs = H Ky^-1 y
  m->LA.assign(kB * kB, 0.0);
  double rhs[kB] = {0, 0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    double h[kB];
    basis(&m->X[(size_t)i * kF], h);
    for (int a = 0; a < kB; ++a) {
      rhs[a] += h[a] * v[i];
      for (int c = 0; c <= a; ++c) m->LA[a * kB + c] += h[a] * m->G[(size_t)c * n + i];
    }
  }
  if (!cholesky(m->LA, kB)) {
    delete m;
    return gadi::set_error(GADI_ERR_INVALID_ARG, "features do not determine the linear mean (rank-deficient basis)");
  }
  std::memcpy(m->b, rhs, sizeof(rhs));
  forward(m->LA, kB, m->b);
  backward(m->LA, kB, m->b);
  // w = Ky^-1 (y - H^T b) = v - G b
  m->w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = v[i];
    for (int j = 0; j < kB; ++j) s -= m->G[(size_t)j * n + i] * m->b[j];
    m->w[i] = s;
  }
  *out = m;
  return GADI_OK;
}

gadi_status gadi_alpha_gpr_predict(const gadi_alpha_gpr* m, const double f[4], double* log10_alpha, double* sd) {
  if (!m || !f || !log10_alpha) return gadi::set_error(GADI_ERR_INVALID_ARG, "null argument");
  for (int i = 0; i < kF; ++i)
    if (!std::isfinite(f[i])) return gadi::set_error(GADI_ERR_INVALID_ARG, "non-finite feature");
  const int n = m->n;
  std::vector<double> ks(n);
  double h[kB];
  basis(f, h);
  double mean = 0.0;
  for (int j = 0; j < kB; ++j) mean += h[j] * m->b[j];
  for (int i = 0; i < n; ++i) {
    ks[i] = m->kern(f, &m->X[(size_t)i * kF]);
    mean += ks[i] * m->w[i];
  }
  *log10_alpha = mean;
  if (sd) {
    // R = h* - H Ky^-1 k* = h* - G^T k*
    double R[kB];
    for (int j = 0; j < kB; ++j) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += m->G[(size_t)j * n + i] * ks[i];
      R[j] = h[j] - s;
    }
    std::vector<double> t(ks);
    forward(m->L, n, t.data());            // k*^T Ky^-1 k* = |L^-1 k*|^2
    double q = 0.0;
    for (int i = 0; i < n; ++i) q += t[i] * t[i];
    double r[kB];
    std::memcpy(r, R, sizeof(R));
    forward(m->LA, kB, r);                 // R^T A^-1 R = |LA^-1 R|^2
    double qa = 0.0;
    for (int j = 0; j < kB; ++j) qa += r[j] * r[j];
    const double var = m->sf2 - q + qa;
    *sd = std::sqrt(var > 0.0 ? var : 0.0);
  }
  return GADI_OK;
}

gadi_status gadi_alpha_gpr_destroy(gadi_alpha_gpr* m) {
  delete m;
  return GADI_OK;
}

}  // extern "C"
