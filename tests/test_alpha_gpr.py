"""Data-driven initial alpha (Section 4.2): features, GPR posterior, packaged model.

CPU: the oracle's features against dense eigenvalues, its GPR posterior
against scikit-learn (zero mean; and the basis-function model through its
equivalent augmented covariance) and against its own limits (interpolation,
generalized least squares), and the C ABI (gadi_alpha_features,
gadi_alpha_gpr_*) against the oracle.  GPU: the packaged model's alpha on
workloads outside its training set.
"""
import ctypes as C
import json
import math
import os

import numpy as np
import pytest

from oracle import gpr, problems
from oracle.problems import hss_split
from paper_2512_21164_amd import _lib, alpha_gpr
from paper_2512_21164_amd.api import Problem

SPECS = [problems.convection_diffusion(2, 9, (3.0, -2.0)),
         problems.convection_diffusion(3, 5, (4.0, 1.0, -6.0)),
         problems.convection_diffusion(2, 8, (10.0, 10.0)),
         problems.complex_reaction_diffusion(7, 30.0)]


def _problem(spec):
    return Problem(spec.dim, tuple(spec.n), spec.center, tuple(spec.lo), tuple(spec.hi),
                   shift_im=spec.shift_im, is_complex=spec.is_complex)


@pytest.mark.parametrize("spec", SPECS)
def test_oracle_features_match_dense_eigenvalues(spec):
    A = problems.assemble(spec)
    M, N = hss_split(A)
    eM = np.linalg.eigvalsh(M.toarray())
    rho = np.max(np.abs(np.linalg.eigvals(N.toarray())))
    for prec, u in (("f32", 2.0 ** -24), ("bf16", 2.0 ** -8), ("f64", 2.0 ** -53)):
        f = gpr.features(spec, prec)
        assert f[0] == pytest.approx(np.log10(eM.min()), abs=1e-12)
        assert f[1] == pytest.approx(np.log10(eM.max()), abs=1e-12)
        assert f[2] == pytest.approx(np.log10(rho), abs=1e-11)
        assert f[3] == np.log10(u)


@pytest.mark.parametrize("spec", SPECS)
def test_c_abi_features_match_oracle(spec):
    for prec in ("f32", "bf16", "f64"):
        assert np.allclose(alpha_gpr.features(_problem(spec), prec), gpr.features(spec, prec), rtol=0, atol=1e-12)


def test_c_abi_features_errors():
    lib = _lib.load()
    f = (C.c_double * 4)()
    st = Problem.convection_diffusion(2, 8, 1.0).c_struct()
    assert lib.gadi_alpha_features(C.byref(st), 7, f) == _lib.GADI_ERR_INVALID_ARG
    assert lib.gadi_alpha_features(None, 0, f) == _lib.GADI_ERR_INVALID_ARG
    indefinite = Problem(2, (8, 8, 1), 1.0, (-1.0, -1.0, 0.0), (-1.0, -1.0, 0.0)).c_struct()
    assert lib.gadi_alpha_features(C.byref(indefinite), 0, f) == _lib.GADI_ERR_UNSUPPORTED


def _data(n=30, seed=0):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(-5, -1, n), rng.uniform(0.5, 1.1, n), rng.uniform(-3, 0, n),
                         rng.choice([np.log10(2.0 ** -24), np.log10(2.0 ** -8)], n)])
    y = 0.5 * (X[:, 0] + X[:, 1]) + 0.1 * np.sin(3 * X[:, 2]) + 0.05 * X[:, 3] + 0.02 * rng.standard_normal(n)
    Xs = np.column_stack([rng.uniform(-6, 0, 7), rng.uniform(0.4, 1.2, 7), rng.uniform(-4, 1, 7),
                          rng.choice([np.log10(2.0 ** -24), np.log10(2.0 ** -8)], 7)])
    return X, y, Xs


HYPER = np.array([1.5, 0.4, 1.2, 2.0, 0.3, 0.05])


def test_oracle_zero_mean_posterior_matches_sklearn():
    from sklearn.gaussian_process import GaussianProcessRegressor
    from sklearn.gaussian_process.kernels import RBF, ConstantKernel
    X, y, Xs = _data()
    ell, sf, sn = HYPER[:4], HYPER[4], HYPER[5]
    gp = GaussianProcessRegressor(ConstantKernel(sf * sf, "fixed") * RBF(ell, "fixed"), alpha=sn * sn,
                                  optimizer=None, normalize_y=False).fit(X, y)
    mu_ref, sd_ref = gp.predict(Xs, return_std=True)
    mu, var = gpr.posterior(X, y, HYPER, Xs, basis_functions=False)
    assert np.allclose(mu, mu_ref, rtol=1e-9, atol=1e-11)
    assert np.allclose(np.sqrt(var), sd_ref, rtol=1e-7, atol=1e-9)


def test_oracle_basis_posterior_matches_augmented_covariance_in_sklearn():
    """A linear mean with a flat prior is the limit b -> inf of a zero-mean GP with covariance
    k(f, f') + b h(f)^T h(f') (Rasmussen and Williams, Section 2.7); sklearn's DotProduct kernel
    on the inputs scaled by sqrt(b) is exactly b h^T h'."""
    from sklearn.gaussian_process import GaussianProcessRegressor
    from sklearn.gaussian_process.kernels import RBF, ConstantKernel, DotProduct
    X, y, Xs = _data(seed=1)
    b = 1e4
    sb = math.sqrt(b)
    ell, sf, sn = HYPER[:4], HYPER[4], HYPER[5]
    kern = ConstantKernel(sf * sf, "fixed") * RBF(ell * sb, "fixed") + DotProduct(sigma_0=sb, sigma_0_bounds="fixed")
    gp = GaussianProcessRegressor(kern, alpha=sn * sn, optimizer=None, normalize_y=False).fit(X * sb, y)
    mu_ref, sd_ref = gp.predict(Xs * sb, return_std=True)
    mu, var = gpr.posterior(X, y, HYPER, Xs)
    assert np.allclose(mu, mu_ref, rtol=1e-5, atol=1e-5)
    assert np.allclose(np.sqrt(var), sd_ref, rtol=1e-3, atol=1e-4)


def test_oracle_posterior_limits():
    X, y, Xs = _data(seed=2)
    # tiny noise: the mean interpolates the data and the variance vanishes there
    h = HYPER.copy(); h[5] = 1e-6
    mu, var = gpr.posterior(X, y, h, X)
    assert np.allclose(mu, y, atol=1e-6)
    assert np.all(var < 1e-8)
    # tiny signal: the mean is the least-squares fit of the linear basis
    h = HYPER.copy(); h[4] = 1e-7
    mu, _ = gpr.posterior(X, y, h, Xs)
    H = np.column_stack([np.ones(len(X)), X])
    coef = np.linalg.lstsq(H, y, rcond=None)[0]
    assert np.allclose(mu, np.column_stack([np.ones(len(Xs)), Xs]) @ coef, atol=1e-9)


def test_c_abi_posterior_matches_oracle():
    X, y, Xs = _data(n=40, seed=3)
    m = alpha_gpr.Model(X, y, HYPER)
    mu_ref, var_ref = gpr.posterior(X, y, HYPER, Xs)
    for i in range(len(Xs)):
        mu, sd = m.predict_features(Xs[i])
        assert mu == pytest.approx(mu_ref[i], rel=1e-10, abs=1e-12)
        assert sd == pytest.approx(math.sqrt(var_ref[i]), rel=1e-7, abs=1e-9)
    m.close()


def test_c_abi_model_errors():
    lib = _lib.load()
    X, y, _ = _data(n=10)
    D = C.POINTER(C.c_double)
    Xc = np.ascontiguousarray(X); yc = np.ascontiguousarray(y)
    h = C.c_void_p()
    bad = np.ascontiguousarray(HYPER.copy()); bad[0] = 0.0
    assert lib.gadi_alpha_gpr_create(10, Xc.ctypes.data_as(D), yc.ctypes.data_as(D), bad.ctypes.data_as(D),
                                     C.byref(h)) == _lib.GADI_ERR_INVALID_ARG
    hy = np.ascontiguousarray(HYPER)
    assert lib.gadi_alpha_gpr_create(5, Xc.ctypes.data_as(D), yc.ctypes.data_as(D), hy.ctypes.data_as(D),
                                     C.byref(h)) == _lib.GADI_ERR_INVALID_ARG
    flat = Xc.copy(); flat[:, 3] = flat[0, 3]          # a constant feature: the linear basis is rank-deficient
    flat = np.ascontiguousarray(flat)
    hy2 = np.ascontiguousarray([1.0, 1.0, 1.0, 1.0, 1e-6, 1e-3])
    assert lib.gadi_alpha_gpr_create(10, flat.ctypes.data_as(D), yc.ctypes.data_as(D), hy2.ctypes.data_as(D),
                                     C.byref(h)) == _lib.GADI_ERR_INVALID_ARG
    assert not h.value


def test_best_alpha_refinement():
    alphas = alpha_gpr.ALPHAS
    la = np.log10(alphas)
    costs = [10 ** ((v + 2.3) ** 2) for v in la]                 # minimum at log10 alpha = -2.3
    assert alpha_gpr.best_log_alpha(alphas, costs) == pytest.approx(-2.3, abs=1e-9)
    costs[0] = math.inf
    assert alpha_gpr.best_log_alpha(alphas, [math.inf] * len(alphas)) is None


def test_packaged_model_is_consistent():
    """The committed model's hyperparameters are a local maximum of the log marginal likelihood
    it was fitted with (to the optimizer's tolerance: no 5% step gains 0.01), and the C ABI
    reproduces the oracle posterior on it."""
    path = alpha_gpr.MODEL_PATH
    if not os.path.exists(path):
        pytest.skip("no packaged model")
    with open(path) as fh:
        m = json.load(fh)
    X, y, hyper = np.array(m["X"]), np.array(m["y"]), np.array(m["hyper"])
    assert X.shape[1] == 4 and len(y) == len(X) >= 20 and len(hyper) == 6
    th = np.log(hyper)
    base = alpha_gpr._log_marginal(th, X, y)
    for i in range(6):
        for d in (-0.05, 0.05):
            t = th.copy(); t[i] += d
            assert alpha_gpr._log_marginal(t, X, y) <= base + 1e-2
    model = alpha_gpr.Model(X, y, hyper)
    mu_ref, _ = gpr.posterior(X, y, hyper, X[:5])
    for i in range(5):
        assert model.predict_features(X[i])[0] == pytest.approx(mu_ref[i], rel=1e-9, abs=1e-10)


@pytest.mark.gpu
def test_gpu_predicted_alpha_is_near_the_best_grid_alpha(gpu_lib):
    """On a problem outside the training set (2D 640^2, beta = 10, FP32 inner solves), the
    packaged model's alpha converges to BE 1e-10 and its algorithmic cost is within 2x of the
    best alpha of the grid within a decade of it."""
    import torch

    import workloads
    from paper_2512_21164_amd import Solver, apply
    pr = Problem.convection_diffusion(2, 640, 10.0)
    a_pred = alpha_gpr.predict_alpha(pr, "f32")
    xt = torch.from_numpy(workloads.x_true(pr.size, 0)).to("cuda")
    b = apply(pr, xt)
    kw = dict(u_s="f32", tol=1e-10, max_outer=6000, inner_tol_h=1e-2, inner_tol_s=1e-2)
    s = Solver(pr, alpha=a_pred, **kw)
    cost = {}
    try:
        grid = [a for a in alpha_gpr.ALPHAS if abs(math.log10(a / a_pred)) <= 1.0]
        for a in [a_pred] + grid:
            s.set_params(alpha=a, **kw)
            _, rep = s.solve(b, torch.zeros_like(b))
            ok = rep["status"] == _lib.GADI_OK
            cost[a] = alpha_gpr.solve_cost(rep, "f32", False) if ok else math.inf
            print(f"alpha {a:.4g}: {rep['status_name']} outer {rep['outer']} cost {cost[a]:.4g}", flush=True)
    finally:
        s.close()
    assert math.isfinite(cost[a_pred])
    assert cost[a_pred] <= 2.0 * min(cost[a] for a in grid)
