"""Gaussian-process regression of the GADI parameter alpha (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 4.2 initialises alpha with a Gaussian-process regression (GPR) model
trained on small problems.  The paper takes its model from a cited work that
is not restated; the reading used here:

* features of a problem: log10 lambda_min(M), log10 lambda_max(M),
  log10 max(rho(N), 1e-12) and log10 u_s, with M, N the Hermitian and
  skew-Hermitian parts of A (closed forms of the stencil) and u_s the unit
  roundoff of Table 1;
* target: log10 of the best alpha of the training problem;
* model: linear mean h(f) = [1, f] with a flat prior on its coefficients,
  squared-exponential covariance with one length scale per feature, and
  Gaussian observation noise.

``posterior`` is the textbook posterior of a GP with explicit basis functions
(Rasmussen and Williams, Gaussian Processes for Machine Learning, 2006,
Section 2.7), written with plain dense solves; ``posterior(..., basis=False)``
is the zero-mean GP of their Section 2.2.
"""
from __future__ import annotations

import numpy as np

from . import closed_forms
from .lowprec import UNIT_ROUNDOFF


def features(spec, prec: str) -> np.ndarray:
    """The four features of a problem (exact eigenvalues of M and N from the Toeplitz closed forms)."""
    eM = closed_forms.eigs_M(spec)
    lmin, lmax = float(eM.min()), float(eM.max())
    if not lmin > 0:
        raise ValueError("M is not positive definite")
    rho = closed_forms.rho_N(spec)
    return np.array([np.log10(lmin), np.log10(lmax), np.log10(max(rho, 1e-12)), np.log10(UNIT_ROUNDOFF[prec])])


def sq_exp(F1, F2, ell, sf) -> np.ndarray:
    """sf^2 exp(-1/2 sum_i ((f_i - f'_i)/ell_i)^2) for all pairs of rows."""
    F1 = np.atleast_2d(F1) / ell
    F2 = np.atleast_2d(F2) / ell
    d2 = ((F1[:, None, :] - F2[None, :, :]) ** 2).sum(axis=2)
    return sf * sf * np.exp(-0.5 * d2)


def basis(F) -> np.ndarray:
    """h(f) = [1, f_0, ..., f_3] as columns (n x 5)."""
    F = np.atleast_2d(F)
    return np.column_stack([np.ones(len(F)), F])


def posterior(X, y, hyper, Fs, basis_functions: bool = True):
    """Posterior mean and variance of the latent function at the rows of Fs.

    hyper = (ell_0, ell_1, ell_2, ell_3, sf, sn).  With basis functions:
        beta = (H Ky^-1 H^T)^-1 H Ky^-1 y,            Ky = K + sn^2 I
        mean = H*^T beta + K*^T Ky^-1 (y - H^T beta)
        var  = k** - K*^T Ky^-1 K* + R^T (H Ky^-1 H^T)^-1 R,   R = H* - H Ky^-1 K*
    (H has one column per training point).  Without: mean = K*^T Ky^-1 y,
    var = k** - K*^T Ky^-1 K*.
    """
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Fs = np.atleast_2d(np.asarray(Fs, dtype=np.float64))
    ell = np.asarray(hyper[:4], dtype=np.float64)
    sf, sn = float(hyper[4]), float(hyper[5])
    Ky = sq_exp(X, X, ell, sf) + sn * sn * np.eye(len(X))
    Ks = sq_exp(X, Fs, ell, sf)                          # n x m
    kss = np.full(len(Fs), sf * sf)
    Kinv_y = np.linalg.solve(Ky, y)
    Kinv_Ks = np.linalg.solve(Ky, Ks)
    if not basis_functions:
        return Ks.T @ Kinv_y, kss - np.sum(Ks * Kinv_Ks, axis=0)
    H = basis(X).T                                       # 5 x n
    Hs = basis(Fs).T                                     # 5 x m
    Kinv_HT = np.linalg.solve(Ky, H.T)                   # n x 5
    A = H @ Kinv_HT
    beta = np.linalg.solve(A, H @ Kinv_y)
    mean = Hs.T @ beta + Ks.T @ np.linalg.solve(Ky, y - H.T @ beta)
    R = Hs - H @ Kinv_Ks
    var = kss - np.sum(Ks * Kinv_Ks, axis=0) + np.sum(R * np.linalg.solve(A, R), axis=0)
    return mean, var
