"""Closed forms for the model problems and dense iteration matrices (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The operators of Section 5 are Kronecker sums of 1-D Toeplitz tridiagonal
matrices.  A Toeplitz tridiagonal T = tridiag(a, d, c) of order m has the
eigenvalues d + 2 sqrt(a c) cos(j pi / (m + 1)), j = 1..m, and the eigenvalues
of a Kronecker sum are the sums of the per-axis eigenvalues.  From this:

* M = (A + A^T)/2 is the h^2-scaled negative Laplacian (plus any reaction
  shift), with eigenvalues  sum_d (c_d + 2 m_d cos theta_{j_d}),
  m_d = (lo_d + hi_d)/2;
* N = (A - A^T)/2 has the eigenvalues  i sum_d (hi_d - lo_d) cos theta_{j_d};
* H = alpha I + M is SPD with kappa(H) = (alpha + lmax) / (alpha + lmin);
* S = alpha I + N is normal with singular values sqrt(alpha^2 + mu^2),
  so kappa(S) = sqrt(alpha^2 + rho(N)^2) / alpha.

The iteration matrix of Section 2.1 is
  T_F(alpha, omega) = (alpha I + N)^{-1} (alpha I + M)^{-1} (alpha^2 I + M N - (1 - omega) alpha A)
and, writing T_PRS = T_F(alpha, 0), T_F = (1 - omega/2) T_PRS + (omega/2) I.
S T_PRS S^{-1} is the product of (alpha I + M)^{-1}(alpha I - M), whose norm is
sigma(alpha) = max_lambda |alpha - lambda| / (alpha + lambda), and a Cayley
transform of the skew N (orthogonal), hence
  rho(T_F) <= (1 - omega/2) sigma(alpha) + omega/2 < 1.
"""
from __future__ import annotations

import itertools

import numpy as np

from .problems import StencilSpec, hss_split, shifted


def toeplitz_eigs(m: int, sub: complex, diag: complex, sup: complex) -> np.ndarray:
    """Eigenvalues of the order-m Toeplitz tridiagonal with constant sub/diag/super."""
    j = np.arange(1, m + 1)
    return diag + 2.0 * np.sqrt(complex(sub) * complex(sup)) * np.cos(j * np.pi / (m + 1))


def _axis_sums(per_axis):
    """All sums of one entry from each per-axis eigenvalue list."""
    return np.array([sum(t) for t in itertools.product(*per_axis)])


def eigs_A(spec: StencilSpec) -> np.ndarray:
    """Eigenvalues of the real stencil operator A (plus i*shift for complex)."""
    c = spec.center / spec.dim
    per = [toeplitz_eigs(spec.n[d], spec.lo[d], c, spec.hi[d]) for d in range(spec.dim)]
    return _axis_sums(per) + 1j * spec.shift_im


def eigs_M(spec: StencilSpec) -> np.ndarray:
    """Eigenvalues of the Hermitian part M (real)."""
    c = spec.center / spec.dim
    per = []
    for d in range(spec.dim):
        m = 0.5 * (spec.lo[d] + spec.hi[d])
        per.append(np.real(toeplitz_eigs(spec.n[d], m, c, m)))
    return np.real(_axis_sums(per))


def eigs_N(spec: StencilSpec) -> np.ndarray:
    """Eigenvalues of the skew-Hermitian part N (purely imaginary)."""
    per = []
    for d in range(spec.dim):
        nu = 0.5 * (spec.hi[d] - spec.lo[d])
        per.append(toeplitz_eigs(spec.n[d], -nu, 0.0, nu))
    return _axis_sums(per) + 1j * spec.shift_im


def lambda_min_max_M(spec: StencilSpec):
    e = eigs_M(spec)
    return float(e.min()), float(e.max())


def rho_N(spec: StencilSpec) -> float:
    """Spectral radius of N."""
    return float(np.max(np.abs(eigs_N(spec))))


def kappa_H(spec: StencilSpec, alpha: float) -> float:
    lmin, lmax = lambda_min_max_M(spec)
    return (alpha + lmax) / (alpha + lmin)


def kappa_S(spec: StencilSpec, alpha: float) -> float:
    r = rho_N(spec)
    return float(np.sqrt(alpha * alpha + r * r) / alpha)


def sigma(spec: StencilSpec, alpha: float) -> float:
    """max over eigenvalues lambda of M of |alpha - lambda| / (alpha + lambda)."""
    e = eigs_M(spec)
    return float(np.max(np.abs(alpha - e) / (alpha + e)))


def alpha_star(spec: StencilSpec) -> float:
    """The alpha minimising sigma(alpha): sqrt(lambda_min * lambda_max)."""
    lmin, lmax = lambda_min_max_M(spec)
    return float(np.sqrt(lmin * lmax))


def contraction_bound(spec: StencilSpec, alpha: float, omega: float) -> float:
    """(1 - omega/2) sigma(alpha) + omega/2, an upper bound on rho(T_F)."""
    return (1.0 - omega / 2.0) * sigma(spec, alpha) + omega / 2.0


def dense_iteration(A, alpha: float, omega: float):
    """Dense T_F(alpha, omega) and the matrix G with x^(k+1) = T_F x^(k) + G b (Section 2.1)."""
    M, N = hss_split(A)
    H, S = shifted(M, N, alpha)
    Md, Nd, Ad = M.toarray(), N.toarray(), A.toarray()
    Hd, Sd = H.toarray(), S.toarray()
    n = Ad.shape[0]
    I = np.eye(n)
    inner = alpha * alpha * I + Md @ Nd - (1.0 - omega) * alpha * Ad
    HS_inv = np.linalg.inv(Sd) @ np.linalg.inv(Hd)      # (alpha I + N)^{-1} (alpha I + M)^{-1}
    TF = HS_inv @ inner
    G = (2.0 - omega) * alpha * HS_inv
    return TF, G


def spectral_radius(T) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(T))))
