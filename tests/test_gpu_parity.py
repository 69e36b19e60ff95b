"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

FP64 parity is checked in "mirror" mode: same b, ||A||, x^(0), alpha, omega and
inner stopping rule on both sides, so the two runs follow the same sequence of
iterates; the tolerance 1e-12 (relative, every compared sweep) is the target
for the GPU FP64 path.  Mixed-precision runs must reach a backward error of
1e-10, recomputed by the oracle in extended precision.
"""
import numpy as np
import pytest

from oracle import gadi_ref, problems
import workloads
from tests._problems import gpu_problem, oracle_system, oracle_system_aniso, rel, to_dev

pytestmark = pytest.mark.gpu

FIXED = dict(tol=0.0, stag_window=0, div_factor=0.0)


def _gpu_solve(spec, b, normA, history=True, x0=None, **kw):
    import torch
    from paper_2512_21164_amd import Solver
    s = Solver(gpu_problem(spec), normA=normA, **kw)
    bd = to_dev(b)
    xd = torch.zeros_like(bd) if x0 is None else to_dev(x0)
    out = s.solve(bd, xd, history=history)
    s.close()
    if history:
        x, rep, hist = out
        return x.cpu().numpy(), rep, hist
    x, rep = out
    return x.cpu().numpy(), rep, None


def test_apply_matches_oracle(gpu_lib):
    from paper_2512_21164_amd import apply
    cases = [problems.convection_diffusion(2, 37, (10.0, -3.0)),
             problems.convection_diffusion(3, 9, (10.0, 2.0, -5.0)),
             problems.complex_reaction_diffusion(21, 10.0)]
    cases.append(oracle_system_aniso(3, (13, 5, 7), (3.0, 4.0, 5.0))[0])
    for spec in cases:
        A = problems.assemble(spec)
        rng = np.random.default_rng(1)
        x = rng.uniform(-1, 1, spec.size)
        if spec.is_complex:
            x = x + 1j * rng.uniform(-1, 1, spec.size)
        for tr in (False, True):
            y = apply(gpu_problem(spec), to_dev(x), transpose=tr).cpu().numpy()
            ref = (A.conj().T if tr else A) @ x
            bound = 1e-15 * 8 * (abs(spec.center) + sum(map(abs, spec.lo)) + sum(map(abs, spec.hi)) + abs(spec.shift_im))
            assert np.max(np.abs(y - ref)) <= bound * np.max(np.abs(x)), (spec, tr)


@pytest.mark.parametrize("dim,ng,beta", [(2, 37, (10.0, -3.0)), (3, 9, (8.0, 8.0, 8.0))])
def test_norm_estimate_is_a_tight_lower_bound(gpu_lib, dim, ng, beta):
    from paper_2512_21164_amd import Solver
    spec, A, x, b = oracle_system(dim, ng, beta)
    exact = gadi_ref.norm2(A)
    s = Solver(gpu_problem(spec))
    est = s.normA
    s.close()
    assert est <= exact * (1 + 1e-12)
    assert est >= exact * (1 - 2e-3)


@pytest.mark.parametrize("omega", [1.0, 0.0])
def test_fixed_iteration_mirror_parity_2d(gpu_lib, omega):
    spec, A, x, b = oracle_system(2, 37, (10.0, -3.0))
    nA = gadi_ref.norm2(A)
    mh, ms = 5, 3
    K = 20
    ref = gadi_ref.gadi(A, b, 0.3, omega, normA=nA, max_outer=K, rule_h=gadi_ref.InnerRule(fixed=mh),
                        rule_s=gadi_ref.InnerRule(fixed=ms), stag_window=0, div_factor=0.0, tol=0.0,
                        record_iterates=True)
    for k in (0, 1, 2, 7, K):
        xg, rep, hist = _gpu_solve(spec, b, nA, alpha=0.3, omega=omega, max_outer=k, fixed_inner_h=mh,
                                   fixed_inner_s=ms, tile_chunk=4, **FIXED)
        assert rep["status"] == gadi_ref.NOT_CONVERGED and rep["outer"] == k
        assert rel(xg, ref.iterates[k]) <= 1e-12 if k else np.all(xg == 0)
        assert np.max(np.abs(hist[:, 0] - np.array(ref.be[: k + 1]))) <= 1e-13
        assert list(hist[:k, 2].astype(int)) == [mh] * k
        assert list(hist[:k, 3].astype(int)) == [ms] * k


def test_fixed_iteration_mirror_parity_3d_ragged(gpu_lib):
    spec, A, x, b = oracle_system_aniso(3, (13, 11, 9), (6.0, -4.0, 9.0))
    nA = gadi_ref.norm2(A)
    ref = gadi_ref.gadi(A, b, 0.4, 1.0, normA=nA, max_outer=12, rule_h=gadi_ref.InnerRule(fixed=4),
                        rule_s=gadi_ref.InnerRule(fixed=2), stag_window=0, div_factor=0.0, tol=0.0,
                        record_iterates=True)
    for ry in (1, 2, 4):
        xg, rep, hist = _gpu_solve(spec, b, nA, alpha=0.4, omega=1.0, max_outer=12, fixed_inner_h=4,
                                   fixed_inner_s=2, tile_ry=ry, tile_chunk=4, **FIXED)
        assert rel(xg, ref.iterates[12]) <= 1e-12, ry
        assert np.max(np.abs(hist[:, 0] - np.array(ref.be))) <= 1e-13


def test_fixed_iteration_mirror_parity_complex(gpu_lib):
    spec = problems.complex_reaction_diffusion(29, 10.0)
    A = problems.assemble(spec)
    b = workloads.complex_rhs(spec.size, 3)
    nA = gadi_ref.norm2(A)
    ref = gadi_ref.gadi(A, b, 0.2, 1.0, normA=nA, max_outer=15, rule_h=gadi_ref.InnerRule(fixed=6),
                        rule_s=gadi_ref.InnerRule(fixed=1), stag_window=0, div_factor=0.0, tol=0.0,
                        record_iterates=True)
    xg, rep, hist = _gpu_solve(spec, b, nA, alpha=0.2, omega=1.0, max_outer=15, fixed_inner_h=6, tile_chunk=4,
                               **FIXED)
    assert rel(xg, ref.iterates[15]) <= 1e-12
    assert np.max(np.abs(hist[:, 0] - np.array(ref.be))) <= 1e-13


def test_c1_parity_to_1e12(gpu_lib):
    """2D convection-diffusion, 64 x 64, alpha 0.5, omega 1, FP64, stop at BE 1e-12."""
    spec, A, x, b = oracle_system(2, 64, (1.0, 1.0), seed=0)
    nA = gadi_ref.norm2(A)
    ref = gadi_ref.gadi(A, b, 0.5, 1.0, normA=nA, tol=1e-12, max_outer=5000)
    xg, rep, hist = _gpu_solve(spec, b, nA, alpha=0.5, omega=1.0, tol=1e-12, max_outer=5000)
    assert rep["status"] == gadi_ref.OK == ref.status
    assert rep["outer"] == ref.outer
    assert list(hist[:-1, 2].astype(int)) == ref.inner_h
    assert list(hist[:-1, 3].astype(int)) == ref.inner_s
    assert rel(xg, ref.x) <= 1e-12
    assert gadi_ref.backward_error(A, xg, b, nA, extended=True) <= 1e-12
    assert gadi_ref.forward_error(xg, x) <= 1e-7


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_precision_reaches_1e10(gpu_lib, prec):
    spec, A, x, b = oracle_system(2, 64, (1.0, 1.0), seed=1)
    nA = gadi_ref.norm2(A)
    xg, rep, hist = _gpu_solve(spec, b, nA, alpha=0.5, omega=1.0, tol=1e-10, u_s=prec, max_outer=5000)
    assert rep["status"] == gadi_ref.OK
    be = gadi_ref.backward_error(A, xg, b, nA, extended=True)
    assert be <= 1e-10 * 1.01
    ref = gadi_ref.gadi(A, b, 0.5, 1.0, normA=nA, tol=1e-10, max_outer=5000, prec=prec)
    assert abs(rep["outer"] - ref.outer) <= 0.05 * ref.outer + 3
    fe = gadi_ref.forward_error(xg, x)
    assert fe <= 1e-5


def test_deterministic_bitwise(gpu_lib):
    spec, A, x, b = oracle_system(2, 100, (20.0, 20.0))
    nA = gadi_ref.norm2(A)
    x1, r1, _ = _gpu_solve(spec, b, nA, alpha=0.1, tol=1e-10, u_s="f32")
    x2, r2, _ = _gpu_solve(spec, b, nA, alpha=0.1, tol=1e-10, u_s="f32")
    assert np.array_equal(x1, x2)
    assert r1["outer"] == r2["outer"] and r1["inner_h"] == r2["inner_h"]


def test_edge_cases(gpu_lib):
    # a single unknown, a single row, max_outer 0, non-zero start
    for spec in (problems.convection_diffusion(2, 1, 1.0), oracle_system_aniso(2, (19, 1), (3.0, 0.0))[0],
                 oracle_system_aniso(3, (1, 1, 7), (0.0, 0.0, 5.0))[0]):
        A = problems.assemble(spec)
        xt = workloads.x_true(spec.size, 4)
        b = A @ xt
        nA = gadi_ref.norm2(A)
        xg, rep, _ = _gpu_solve(spec, b, nA, alpha=0.5, tol=1e-12, max_outer=5000)
        assert rep["status"] == gadi_ref.OK
        assert gadi_ref.backward_error(A, xg, b, nA, extended=True) <= 1e-12
    spec, A, x, b = oracle_system(2, 16, (2.0, 2.0))
    nA = gadi_ref.norm2(A)
    x0 = workloads.x_true(spec.size, 9)
    xg, rep, hist = _gpu_solve(spec, b, nA, x0=x0, alpha=0.5, max_outer=0)
    assert rep["status"] == gadi_ref.NOT_CONVERGED and np.array_equal(xg, x0)
    assert abs(hist[0, 0] - gadi_ref.backward_error(A, x0, b, nA)) <= 1e-15
    # b = 0: the zero start is the exact solution (backward error 0, not 0 / 0), as in the oracle
    z = np.zeros_like(b)
    ref = gadi_ref.gadi(A, z, 0.5, 1.0, normA=nA, tol=1e-12, max_outer=10)
    xg, rep, hist = _gpu_solve(spec, z, nA, alpha=0.5, tol=1e-12, max_outer=10)
    assert rep["status"] == ref.status == gadi_ref.OK and rep["outer"] == ref.outer == 0
    assert hist[0, 0] == 0.0 and not np.any(xg)


def test_status_codes(gpu_lib):
    spec, A, x, b = oracle_system(2, 16, (10.0, 5.0))
    nA = gadi_ref.norm2(A)
    _, rep, _ = _gpu_solve(spec, b, nA, alpha=0.5, max_outer=1)
    assert rep["status"] == gadi_ref.NOT_CONVERGED and rep["outer"] == 1
    _, rep, _ = _gpu_solve(spec, b, nA, alpha=1e5, max_outer=100, stag_window=5)
    ref = gadi_ref.gadi(A, b, 1e5, 1.0, normA=nA, max_outer=100, stag_window=5)
    assert rep["status"] == gadi_ref.STAGNATED == ref.status and rep["outer"] == ref.outer
    bn = b.copy()
    bn[3] = np.nan
    _, rep, _ = _gpu_solve(spec, bn, nA, alpha=0.5, max_outer=10)
    assert rep["status"] == gadi_ref.DIVERGED and rep["outer"] == 0


def test_async_solve_matches_blocking(gpu_lib):
    import torch
    from paper_2512_21164_amd import Solver
    spec, A, x, b = oracle_system(2, 48, (5.0, 5.0))
    nA = gadi_ref.norm2(A)
    xb, rb, _ = _gpu_solve(spec, b, nA, alpha=0.3, u_s="f32")
    s = Solver(gpu_problem(spec), normA=nA, alpha=0.3, u_s="f32")
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    s.solve_async(bd, xd)
    rep = None
    for _ in range(100000):
        rep = s.query(wait=False)
        if rep is not None:
            break
    assert rep is not None and rep["status"] == 0
    assert np.array_equal(xd.cpu().numpy(), xb)
    s.close()
