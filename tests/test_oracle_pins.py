"""Pins of the CPU oracle against closed forms and identities of the paper.

Every check here compares the oracle with something other than itself: the
analytic spectrum of Toeplitz Kronecker sums, exactness of centered
differences on polynomials, the two-step form of Section 2.1 against the
four-step Algorithm 1, the iteration matrix T_F and the (HS)^{-1} identity of
Section 3.2, Lemma 1 and the contraction bound, Remark 1, the backward-error
characterisation of Section 3, dense LU solves, and finite termination of CG.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import closed_forms as cf
from oracle import gadi_ref, problems


def _match_multiset(a, b, tol):
    a = np.sort_complex(np.asarray(a, dtype=complex))
    b = np.asarray(b, dtype=complex)
    used = np.zeros(len(b), bool)
    for v in a:
        d = np.abs(b - v)
        d[used] = np.inf
        k = int(np.argmin(d))
        assert d[k] <= tol, (v, b[k])
        used[k] = True


@pytest.mark.parametrize("spec", [
    problems.convection_diffusion(2, 6, (3.0, -2.0)),
    problems.convection_diffusion(2, 7, (30.0, 5.0), reaction=100.0),
    problems.convection_diffusion(3, 4, (6.0, 1.0, -4.0)),
    problems.complex_reaction_diffusion(6, 10.0),
])
def test_spectrum_matches_toeplitz_closed_form(spec):
    A = problems.assemble(spec).toarray()
    _match_multiset(np.linalg.eigvals(A), cf.eigs_A(spec), 1e-10)
    M, N = problems.hss_split(problems.assemble(spec))
    _match_multiset(np.linalg.eigvalsh(M.toarray()), cf.eigs_M(spec), 1e-10)
    _match_multiset(np.linalg.eigvals(N.toarray()), cf.eigs_N(spec), 1e-10)


def test_eigenvectors_fix_axis_order():
    """Tensor products of the 1-D Toeplitz eigenvectors are eigenvectors of A.

    Different convection per axis makes a transposed axis order fail.
    """
    spec = problems.convection_diffusion(3, 5, (8.0, -7.0, 3.0))
    A = problems.assemble(spec)
    c = spec.center / spec.dim
    vecs, vals = [], []
    for d in range(3):
        m = spec.n[d]
        a, cc = spec.lo[d], spec.hi[d]
        i = np.arange(1, m + 1)
        j = 2
        th = j * np.pi / (m + 1)
        rr = np.sqrt(a / cc)
        vecs.append(rr ** i * np.sin(i * th))
        vals.append(c + (a / rr + cc * rr) * np.cos(th))
    v = np.einsum("k,j,i->kji", vecs[2], vecs[1], vecs[0]).ravel()
    lam = sum(vals)
    assert np.linalg.norm(A @ v - lam * v) <= 1e-12 * np.linalg.norm(v) * abs(lam)


@pytest.mark.parametrize("dim", [2, 3])
def test_centered_differences_exact_on_quadratics(dim):
    """A u_h = h^2 (-Lap u + beta.grad u + c u) at the nodes for u quadratic per axis.

    Centered first and second differences are exact for quadratics, and
    u = prod x_d (1 - x_d) vanishes on the boundary, so the identity is exact.
    This fixes the sign of the convection term and the h^2 scaling.
    """
    ng, beta, react = 9, (7.0, -3.0, 5.0)[:dim], 11.0
    spec = problems.convection_diffusion(dim, ng, beta, reaction=react)
    A = problems.assemble(spec)
    h = 1.0 / (ng + 1)
    if dim == 2:
        u = lambda X, Y: X * (1 - X) * Y * (1 - Y)
        pde = lambda X, Y: (2 * Y * (1 - Y) + 2 * X * (1 - X)
                            + beta[0] * (1 - 2 * X) * Y * (1 - Y)
                            + beta[1] * X * (1 - X) * (1 - 2 * Y)
                            + react * X * (1 - X) * Y * (1 - Y))
    else:
        q = lambda t: t * (1 - t)
        dq = lambda t: 1 - 2 * t
        u = lambda X, Y, Z: q(X) * q(Y) * q(Z)
        pde = lambda X, Y, Z: (2 * q(Y) * q(Z) + 2 * q(X) * q(Z) + 2 * q(X) * q(Y)
                               + beta[0] * dq(X) * q(Y) * q(Z)
                               + beta[1] * q(X) * dq(Y) * q(Z)
                               + beta[2] * q(X) * q(Y) * dq(Z)
                               + react * q(X) * q(Y) * q(Z))
    lhs = A @ problems.grid_function(spec, u)
    rhs = h * h * problems.grid_function(spec, pde)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14 * np.max(np.abs(rhs)) * 10


def test_hss_split_properties():
    for spec in (problems.convection_diffusion(2, 5, (4.0, 9.0)),
                 problems.complex_reaction_diffusion(5, 3.0)):
        A = problems.assemble(spec)
        M, N = problems.hss_split(A)
        assert abs(M - M.conj().T).max() == 0
        assert abs(N + N.conj().T).max() == 0
        assert abs(M + N - A).max() <= 1e-15


def _small_system(ng=8, beta=(10.0, 5.0), seed=3):
    spec = problems.convection_diffusion(2, ng, beta)
    A = problems.assemble(spec)
    x = workloads.x_true(spec.size, seed)
    return spec, A, x, A @ x


@pytest.mark.parametrize("omega", [0.0, 0.7, 1.0, 1.5])
def test_two_step_form_equals_algorithm1(omega):
    """Section 2.1's two-step GADI and Algorithm 1 (exact solves) give the same iterates."""
    spec, A, x, b = _small_system()
    res = gadi_ref.gadi(A, b, 0.3, omega, normA=gadi_ref.norm2(A), tol=0.0, max_outer=12,
                        inner="exact", stag_window=0, record_iterates=True)
    two = gadi_ref.gadi_two_step(A, b, 0.3, omega, 12)
    for k in range(13):
        ref = two[k]
        den = max(np.linalg.norm(ref), 1e-300)
        assert np.linalg.norm(res.iterates[k] - ref) <= 1e-12 * den + (0 if k else 0)


@pytest.mark.parametrize("alpha,omega", [(0.05, 0.0), (0.3, 1.0), (2.0, 1.6)])
def test_iteration_matrix_drives_iterates(alpha, omega):
    """x^(k+1) = T_F x^(k) + G b with T_F, G of Section 2.1 (dense)."""
    spec, A, x, b = _small_system(ng=6, beta=(12.0, -4.0))
    TF, G = cf.dense_iteration(A, alpha, omega)
    res = gadi_ref.gadi(A, b, alpha, omega, normA=1.0, tol=0.0, max_outer=8, inner="exact",
                        stag_window=0, record_iterates=True)
    for k in range(8):
        pred = TF @ res.iterates[k] + G @ b
        assert np.linalg.norm(res.iterates[k + 1] - pred) <= 1e-12 * np.linalg.norm(pred)


def test_hs_inverse_identity():
    """(HS)^{-1} = (I - T_F) A^{-1} / (alpha (2 - omega)), used in the proof of Theorem 2."""
    spec, A, x, b = _small_system(ng=5, beta=(8.0, 3.0))
    alpha, omega = 0.4, 0.6
    TF, _ = cf.dense_iteration(A, alpha, omega)
    M, N = problems.hss_split(A)
    H, S = problems.shifted(M, N, alpha)
    lhs = np.linalg.inv(H.toarray() @ S.toarray())
    rhs = (np.eye(A.shape[0]) - TF) @ np.linalg.inv(A.toarray()) / (alpha * (2 - omega))
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))


@pytest.mark.parametrize("spec", [problems.convection_diffusion(2, 6, (20.0, 20.0)),
                                  problems.convection_diffusion(3, 3, (5.0, 5.0, 5.0)),
                                  problems.complex_reaction_diffusion(5, 50.0)])
def test_lemma1_and_contraction_bound(spec):
    """rho(T_F) < 1 for all alpha > 0, omega in [0,2) (Lemma 1) and the Cayley bound."""
    A = problems.assemble(spec)
    for alpha in (1e-2, 0.1, 1.0, 10.0):
        for omega in (0.0, 0.5, 1.0, 1.9):
            rho = cf.spectral_radius(cf.dense_iteration(A, alpha, omega)[0])
            assert rho < 1.0
            assert rho <= cf.contraction_bound(spec, alpha, omega) + 1e-12


def test_asymptotic_rate_tends_to_spectral_radius():
    """Remark 1: the per-sweep error reduction tends to rho(T_F)."""
    spec, A, x, b = _small_system(ng=8, beta=(3.0, 3.0))
    alpha, omega = 0.2, 1.0
    rho = cf.spectral_radius(cf.dense_iteration(A, alpha, omega)[0])
    res = gadi_ref.gadi(A, b, alpha, omega, normA=1.0, tol=0.0, max_outer=60, inner="exact",
                        stag_window=0, record_iterates=True)
    e = [np.linalg.norm(v - x) for v in res.iterates]
    rate = (e[60] / e[40]) ** (1.0 / 20)
    assert abs(rate - rho) <= 0.02 * rho


def test_backward_error_at_zero_start_is_one():
    spec, A, x, b = _small_system()
    res = gadi_ref.gadi(A, b, 0.5, 1.0, normA=gadi_ref.norm2(A), tol=0.0, max_outer=0)
    assert res.be[0] == 1.0
    assert res.status == gadi_ref.NOT_CONVERGED


def test_backward_error_is_realised_by_a_perturbation():
    """The BE formula of Section 3 is attained by the rank-one (Rigal-Gaches) perturbation."""
    spec, A, x, b = _small_system(ng=5)
    rng = np.random.default_rng(7)
    xh = x + 1e-3 * rng.standard_normal(x.size)
    nA = gadi_ref.norm2(A)
    eps = gadi_ref.backward_error(A, xh, b, nA)
    r = b - A @ xh
    nx, nb = np.linalg.norm(xh), np.linalg.norm(b)
    den = nA * nx + nb
    dA = (nA * nx / den) * np.outer(r, xh) / nx ** 2
    db = -(nb / den) * r
    assert np.allclose((A.toarray() + dA) @ xh, b + db, rtol=0, atol=1e-13)
    assert abs(np.linalg.norm(dA, 2) - eps * nA) <= 1e-12 * eps * nA
    assert abs(np.linalg.norm(db) - eps * nb) <= 1e-12 * eps * nb
    assert abs(gadi_ref.backward_error(A, xh, b, nA, extended=True) - eps) <= 1e-12 * eps


def test_backward_error_of_an_exact_solution_is_zero():
    """The backward error is the smallest relative perturbation of A and b that x solves exactly
    (Section 3); an exact x needs none, so it is 0, also for b = 0 and x = 0 where the quotient
    of the formula is 0 / 0.  With b = 0 the zero start is that exact solution: GADI stops at
    sweep 0 with status OK instead of reading 0 / 0 as a non-finite (diverged) backward error."""
    spec, A, x, b = _small_system(ng=6)
    nA = gadi_ref.norm2(A)
    z = np.zeros_like(b)
    assert gadi_ref.backward_error(A, z, z, nA) == 0.0
    assert gadi_ref.backward_error(A, z, z, nA, extended=True) == 0.0
    assert gadi_ref.backward_error_stencil(spec, z, z, nA) == 0.0
    s0, A0, x0, _ = _small_system(ng=6, beta=(0.0, 0.0))   # integer stencil: -1 and 4
    xd = np.round(x0 * 8) / 8                               # dyadic, so A0 xd is exact in FP64
    assert gadi_ref.backward_error(A0, xd, A0 @ xd, gadi_ref.norm2(A0), extended=True) == 0.0
    res = gadi_ref.gadi(A, z, 0.5, 1.0, normA=nA, tol=1e-12, max_outer=10)
    assert res.status == gadi_ref.OK and res.outer == 0 and res.be == [0.0]
    assert not np.any(res.x)
    # a non-zero start with b = 0 has a finite, positive backward error (x = 0 is the solution)
    res = gadi_ref.gadi(A, z, 0.5, 1.0, normA=nA, x0=x, tol=0.0, max_outer=0)
    assert 0.0 < res.be[0] <= 1.0


@pytest.mark.parametrize("ng,beta,alpha", [(8, (1.0, 1.0), 0.5), (12, (30.0, 10.0), 0.2),
                                           (16, (5.0, 50.0), 0.1)])
def test_converged_solution_matches_dense_lu(ng, beta, alpha):
    spec = problems.convection_diffusion(2, ng, beta)
    A = problems.assemble(spec)
    x = workloads.x_true(spec.size, 1)
    b = A @ x
    nA = gadi_ref.norm2(A)
    res = gadi_ref.gadi(A, b, alpha, 1.0, normA=nA, tol=1e-13, max_outer=20000)
    assert res.status == gadi_ref.OK
    xd = np.linalg.solve(A.toarray(), b)
    kappa = np.linalg.cond(A.toarray(), 2)
    be = gadi_ref.backward_error(A, res.x, b, nA, extended=True)
    assert be <= 1e-13
    assert gadi_ref.forward_error(res.x, xd) <= 2 * kappa * be + 1e-14


def test_3d_converges_to_dense_solution():
    spec = problems.convection_diffusion(3, 6, (10.0, 10.0, 10.0))
    A = problems.assemble(spec)
    x = workloads.x_true(spec.size, 2, "normal")
    b = A @ x
    nA = gadi_ref.norm2(A)
    res = gadi_ref.gadi(A, b, 0.3, 1.0, normA=nA, tol=1e-12, max_outer=5000)
    assert res.status == gadi_ref.OK
    assert gadi_ref.forward_error(res.x, np.linalg.solve(A.toarray(), b)) <= 1e-9


def test_cg_terminates_within_distinct_eigenvalues():
    spec = problems.convection_diffusion(2, 4, (0.0, 0.0))
    A = problems.assemble(spec)
    M, N = problems.hss_split(A)
    H, _ = problems.shifted(M, N, 0.5)
    distinct = len(np.unique(np.round(cf.eigs_M(spec) + 0.5, 10)))
    c = workloads.x_true(spec.size, 5)
    rule = gadi_ref.InnerRule(tol=1e-13, max_iter=100, stag_window=0)
    z, it = gadi_ref.cg(H, c, rule, "f64")
    assert it <= distinct
    assert np.linalg.norm(c - H @ z) <= 1e-13 * np.linalg.norm(c)


def test_cg_recursive_residual_tracks_true_residual():
    spec = problems.convection_diffusion(2, 10, (5.0, 5.0))
    M, N = problems.hss_split(problems.assemble(spec))
    H, _ = problems.shifted(M, N, 0.05)
    c = workloads.x_true(spec.size, 6)
    for m in (1, 3, 10):
        z, it = gadi_ref.cg(H, c, gadi_ref.InnerRule(fixed=m), "f64")
        assert it == m
        # the relative residual of the fixed-iteration solve decreases with m
    z1, _ = gadi_ref.cg(H, c, gadi_ref.InnerRule(tol=1e-8, stag_window=0), "f64")
    assert np.linalg.norm(c - H @ z1) <= 1.01e-8 * np.linalg.norm(c)


def test_cgne_solves_shifted_skew_system():
    spec = problems.convection_diffusion(2, 10, (40.0, -25.0))
    M, N = problems.hss_split(problems.assemble(spec))
    _, S = problems.shifted(M, N, 0.01)
    c = workloads.x_true(spec.size, 8)
    y, it = gadi_ref.cgne(S, c, gadi_ref.InnerRule(tol=1e-12, stag_window=0), "f64")
    ys = sp.linalg.spsolve(sp.csc_matrix(S), c)
    assert np.linalg.norm(y - ys) <= 1e-10 * np.linalg.norm(ys)
    assert it < spec.size


def test_cgne_on_constant_complex_shift_takes_one_iteration():
    spec = problems.complex_reaction_diffusion(8, 10.0)
    M, N = problems.hss_split(problems.assemble(spec))
    _, S = problems.shifted(M, N, 0.3)
    c = workloads.complex_rhs(spec.size, 1)
    y, it = gadi_ref.cgne(S, c, gadi_ref.InnerRule(tol=1e-14, stag_window=0), "f64")
    assert it == 1
    assert np.max(np.abs(y - c / (0.3 + 1j * spec.shift_im))) <= 1e-15 * np.max(np.abs(y))


def test_complex_form_equals_real_block_form():
    """Section 5.4 solves the real block form; the Hermitian split of the complex form matches."""
    spec = problems.complex_reaction_diffusion(6, 2000.0)
    A = problems.assemble(spec)
    b = workloads.complex_rhs(spec.size, 4)
    Ab = problems.real_block_form(A)
    bb = np.concatenate([b.real, b.imag])
    nA = gadi_ref.norm2(Ab)
    rc = gadi_ref.gadi(A, b, 0.2, 1.0, normA=nA, tol=0.0, max_outer=10, inner="exact",
                       stag_window=0, record_iterates=True)
    rb = gadi_ref.gadi(Ab, bb, 0.2, 1.0, normA=nA, tol=0.0, max_outer=10, inner="exact",
                       stag_window=0, record_iterates=True)
    n = spec.size
    for k in range(11):
        xc = rc.iterates[k]
        xb = rb.iterates[k][:n] + 1j * rb.iterates[k][n:]
        assert np.linalg.norm(xc - xb) <= 1e-12 * max(np.linalg.norm(xb), 1e-300)
    assert np.allclose(rc.be, rb.be, rtol=1e-10, atol=1e-16)


def test_status_rules():
    spec, A, x, b = _small_system()
    nA = gadi_ref.norm2(A)
    r = gadi_ref.gadi(A, b, 0.5, 1.0, normA=nA, tol=1e-10, max_outer=1)
    assert r.status == gadi_ref.NOT_CONVERGED and r.outer == 1
    # a huge alpha makes T_F close to the identity: no 1% progress in 5 sweeps
    r = gadi_ref.gadi(A, b, 1e5, 1.0, normA=nA, tol=1e-10, max_outer=100, stag_window=5)
    assert r.status == gadi_ref.STAGNATED and r.outer == 5
    bn = b.copy()
    bn[3] = np.nan
    r = gadi_ref.gadi(A, bn, 0.5, 1.0, normA=nA, tol=1e-10, max_outer=10)
    assert r.status == gadi_ref.DIVERGED and r.outer == 0
    r = gadi_ref.gadi(A, b, 0.5, 1.0, normA=nA, tol=1e-10, max_outer=10000)
    assert r.status == gadi_ref.OK
    with pytest.raises(ValueError):
        gadi_ref.gadi(A, b, 0.0, 1.0, normA=nA)
    with pytest.raises(ValueError):
        gadi_ref.gadi(A, b, 0.5, 2.0, normA=nA)
