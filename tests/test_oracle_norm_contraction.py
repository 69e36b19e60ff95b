"""Pins of the oracle's 2-norm of A and of its contraction closed forms.

The backward error of Section 3 divides by ||A||_2, and every parity test
passes the oracle's ``norm2`` to both sides, so a wrong 2-norm would go
unnoticed by them: it is pinned here on its own.  ``norm2`` takes a dense SVD
up to 1024 unknowns and ARPACK (``svds``) above; the ARPACK branch is checked
against

* a dense SVD of the same matrix (grids just above the switch, with
  convection, in 2D and 3D);
* the closed form lambda_max(M) when beta = 0 (A = M is symmetric, so its
  2-norm is its largest eigenvalue, a Toeplitz Kronecker-sum closed form);
* the two-sided bound lambda_max(M) <= ||A||_2 <= lambda_max(M) + rho(N) for
  A = M + N with M symmetric and N skew (x^T A x = x^T M x gives the lower
  bound, the triangle inequality and ||N||_2 = rho(N) for a normal N the upper
  one), both ends closed forms, and max |lambda(A)| <= ||A||_2, on the 64^2
  parity grid.

sigma(alpha) is checked against a brute-force maximum over the dense
eigenvalues of M, two-sidedly through rho(T_PRS) = sigma(alpha) when N = 0
(then (alpha I + M)^{-1} (alpha I - M) is the whole iteration matrix at
omega = 0, and it is symmetric), and alpha* = sqrt(lambda_min lambda_max)
against a brute-force minimum of sigma over a fine alpha grid.
"""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import gadi_ref, problems


@pytest.mark.parametrize("spec", [
    problems.convection_diffusion(2, 33, (10.0, -4.0)),          # 1089 unknowns
    problems.convection_diffusion(2, 40, (100.0, 100.0)),        # cell Peclet 1.2 in x and y
    problems.convection_diffusion(3, 11, (10.0, 10.0, 10.0)),    # 1331 unknowns
    problems.complex_reaction_diffusion(36, 10.0),               # 1296 complex unknowns
])
def test_norm2_arpack_branch_equals_dense_svd(spec):
    A = problems.assemble(spec)
    assert A.shape[0] > 1024, "the grid must exercise the ARPACK branch"
    dense = float(np.linalg.svd(A.toarray(), compute_uv=False)[0])
    assert abs(gadi_ref.norm2(A) - dense) <= 1e-12 * dense


@pytest.mark.parametrize("dim,ng", [(2, 40), (3, 12)])
def test_norm2_symmetric_equals_lambda_max(dim, ng):
    spec = problems.convection_diffusion(dim, ng, (0.0,) * dim)
    A = problems.assemble(spec)
    assert A.shape[0] > 1024
    lmax = cf.lambda_min_max_M(spec)[1]
    # lambda_max(M) = d * 4 cos^2(pi / (2 (ng + 1))) for the h^2-scaled Laplacian
    assert abs(lmax - dim * 4.0 * np.cos(np.pi / (2 * (ng + 1))) ** 2) <= 1e-13 * lmax
    assert abs(gadi_ref.norm2(A) - lmax) <= 1e-12 * lmax


def test_norm2_parity_grid_between_closed_form_bounds():
    spec = problems.convection_diffusion(2, 64, (1.0, 1.0))
    A = problems.assemble(spec)
    nA = gadi_ref.norm2(A)
    lmin, lmax = cf.lambda_min_max_M(spec)
    rho = cf.rho_N(spec)
    lam_A = np.max(np.abs(cf.eigs_A(spec)))
    assert lmax - 1e-12 <= nA <= lmax + rho + 1e-12
    assert lam_A <= nA + 1e-12
    # the value the parity configuration quotes
    assert abs(nA - 7.995329) <= 5e-7


@pytest.mark.parametrize("spec", [problems.convection_diffusion(2, 7, (3.0, 3.0)),
                                  problems.convection_diffusion(3, 4, (1.0, 2.0, 3.0)),
                                  problems.convection_diffusion(2, 9, (0.0, 0.0), reaction=50.0)])
def test_sigma_equals_brute_force_over_dense_spectrum(spec):
    M, _ = problems.hss_split(problems.assemble(spec))
    lam = np.linalg.eigvalsh(M.toarray())
    for alpha in (1e-3, 0.05, 0.4, 3.0, 40.0):
        brute = max(abs(alpha - l) / (alpha + l) for l in lam)
        assert abs(cf.sigma(spec, alpha) - brute) <= 1e-13
        for omega in (0.0, 1.0, 1.99):
            assert cf.contraction_bound(spec, alpha, omega) < 1.0


@pytest.mark.parametrize("dim,ng", [(2, 6), (3, 3)])
def test_prs_radius_equals_sigma_without_convection(dim, ng):
    """beta = 0: N = 0, T_F(alpha, 0) = (alpha I + M)^{-1}(alpha I - M), rho = sigma exactly."""
    spec = problems.convection_diffusion(dim, ng, (0.0,) * dim)
    A = problems.assemble(spec)
    for alpha in (0.01, 0.3, 2.0):
        rho = cf.spectral_radius(cf.dense_iteration(A, alpha, 0.0)[0])
        assert abs(rho - cf.sigma(spec, alpha)) <= 1e-12
        # and the omega-bound is attained as well: with N = 0 the eigenvalues of T_F are
        # (1 - omega/2) (alpha - l)/(alpha + l) + omega/2, the largest in modulus at the
        # smallest l for alpha > l_min
        rho1 = cf.spectral_radius(cf.dense_iteration(A, alpha, 1.0)[0])
        lam = cf.eigs_M(spec)
        assert abs(rho1 - np.max(np.abs(0.5 * (alpha - lam) / (alpha + lam) + 0.5))) <= 1e-12


def test_alpha_star_minimises_sigma():
    spec = problems.convection_diffusion(2, 64, (1.0, 1.0))
    a_star = cf.alpha_star(spec)
    assert abs(a_star - 0.1933) <= 5e-4      # sqrt(4.671e-3 * 7.9953)
    grid = np.logspace(-3, 1, 2001)
    s_grid = np.array([cf.sigma(spec, a) for a in grid])
    s_star = cf.sigma(spec, a_star)
    assert s_star <= s_grid.min() + 1e-12
    assert abs(grid[np.argmin(s_grid)] / a_star - 1.0) <= 0.01
