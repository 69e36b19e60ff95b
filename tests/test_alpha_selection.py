"""Alpha selection of Section 4.3 (safeguard, step 2; restarts, step 3).

CPU checks of the oracle procedure against dense linear algebra and its own
invariants, and of the library's host-side condition estimate.  The GPU
check compares the library's restarting solve with the oracle's.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import gadi_ref, problems
from oracle.lowprec import UNIT_ROUNDOFF
from oracle.problems import hss_split, shifted
from tests._problems import gpu_problem, oracle_system, rel, to_dev

G = gadi_ref.ALPHA_GROWTH

# grids of odd size: N then has a zero eigenvalue and kappa(S) is exact
SPECS = [problems.convection_diffusion(2, 7, (3.0, -2.0)),
         problems.convection_diffusion(3, 5, (4.0, 1.0, -6.0)),
         problems.convection_diffusion(2, 9, (0.0, 0.0), reaction=3.0)]


def dense_kappas(spec, alpha):
    A = problems.assemble(spec)
    M, N = hss_split(A)
    H, S = shifted(M, N, alpha)
    return np.linalg.cond(H.toarray(), 2), np.linalg.cond(S.toarray(), 2)


@pytest.mark.parametrize("spec", SPECS)
def test_safeguard_picks_first_grid_alpha_meeting_the_dense_condition(spec):
    """Brute force over alpha * G^m with dense 2-norm condition numbers."""
    for prec, tau, a0 in (("bf16", 0.01, 1e-3), ("bf16", 0.5, 1e-2), ("f32", 1e-4, 1e-3), ("f64", 1e-12, 1e-4)):
        u = UNIT_ROUNDOFF[prec]
        a, m = a0, 0
        while True:
            kh, ks = dense_kappas(spec, a)
            if kh * ks * u < tau:
                break
            a *= G
            m += 1
            assert m < 200
        assert gadi_ref.safeguarded_alpha(spec, a0, prec, tau) == pytest.approx(a, rel=1e-12)


def test_safeguard_off_and_invalid_tau():
    spec = SPECS[0]
    assert gadi_ref.safeguarded_alpha(spec, 0.123, "bf16", 0.0) == 0.123
    with pytest.raises(ValueError):
        gadi_ref.safeguarded_alpha(spec, 0.1, "bf16", 1e-3)     # tau below the unit roundoff of BF16


def _stagnating_case():
    spec, A, x, b = oracle_system(2, 15, (1.0, 1.0), seed=0)
    return spec, A, x, b, gadi_ref.norm2(A)


def test_restarts_rescue_a_stagnating_solve():
    spec, A, x, b, nA = _stagnating_case()
    kw = dict(tol=1e-12, stag_window=5)
    plain = gadi_ref.gadi(A, b, 1e-4, 1.0, normA=nA, max_outer=3000, **kw)
    assert plain.status == gadi_ref.STAGNATED
    r = gadi_ref.gadi_select_alpha(A, b, 1e-4, 1.0, spec=spec, normA=nA, max_outer=3000, max_restarts=12, **kw)
    assert r.status == gadi_ref.OK and r.restarts >= 2
    assert r.alpha == pytest.approx(1e-4 * G ** r.restarts, rel=1e-12)
    assert r.outer == sum(t.outer for t in r.attempts) <= 3000
    assert all(t.status == gadi_ref.STAGNATED for t in r.attempts[:-1])
    # each attempt resumes from the previous attempt's iterate: its first BE is the previous last BE
    for prev, nxt in zip(r.attempts, r.attempts[1:]):
        assert nxt.be[0] == pytest.approx(prev.be[-1], rel=1e-12)
    assert gadi_ref.backward_error(A, r.x, b, nA, extended=True) <= 1e-12
    assert gadi_ref.forward_error(r.x, x) <= 1e-6


def test_restart_after_divergence_starts_from_zero():
    spec, A, x, b, nA = _stagnating_case()
    # with omega = 0 the BE grows by ~19% at sweep 2: a divergence factor of 1.1 stops there
    r = gadi_ref.gadi_select_alpha(A, b, 1.0, 0.0, spec=spec, normA=nA, tol=1e-12, max_outer=400,
                                   max_restarts=1, div_factor=1.1)
    assert r.attempts[0].status == gadi_ref.DIVERGED
    assert r.restarts == 1
    assert r.attempts[1].be[0] == pytest.approx(1.0, rel=1e-15)     # x = 0: BE = ||b|| / ||b||


def test_restart_budget_is_shared():
    spec, A, x, b, nA = _stagnating_case()
    r = gadi_ref.gadi_select_alpha(A, b, 1e-4, 1.0, spec=spec, normA=nA, tol=1e-12, max_outer=150,
                                   stag_window=5, max_restarts=12)
    assert r.outer == sum(t.outer for t in r.attempts) <= 150


# ---------------------------------------------------------------- C ABI (host only)
def test_condition_estimate_matches_dense():
    from paper_2512_21164_amd import _lib
    lib = _lib.load()
    cases = SPECS + [problems.complex_reaction_diffusion(7, 10.0)]
    for spec in cases:
        st = gpu_problem(spec).c_struct()
        for alpha in (1e-3, 0.05, 0.7, 3.0):
            kh, ks = C.c_double(), C.c_double()
            assert lib.gadi_condition_estimate(C.byref(st), alpha, C.byref(kh), C.byref(ks)) == 0
            dh, ds = dense_kappas(spec, alpha)
            assert kh.value == pytest.approx(dh, rel=1e-10), (spec, alpha)
            if spec.shift_im == 0.0:
                assert ks.value == pytest.approx(ds, rel=1e-10), (spec, alpha)
            else:   # constant imaginary shift: S is a multiple of I, the estimate is an upper bound
                assert ds == pytest.approx(1.0, rel=1e-12) and ks.value >= ds


def test_condition_estimate_errors():
    from paper_2512_21164_amd import _lib
    lib = _lib.load()
    st = gpu_problem(SPECS[0]).c_struct()
    kh, ks = C.c_double(), C.c_double()
    assert lib.gadi_condition_estimate(C.byref(st), 0.0, C.byref(kh), C.byref(ks)) == _lib.GADI_ERR_INVALID_ARG
    assert lib.gadi_condition_estimate(C.byref(st), 0.1, None, C.byref(ks)) == _lib.GADI_ERR_INVALID_ARG
    st.dim = 4
    assert lib.gadi_condition_estimate(C.byref(st), 0.1, C.byref(kh), C.byref(ks)) == _lib.GADI_ERR_INVALID_ARG


# ---------------------------------------------------------------- GPU
@pytest.mark.gpu
def test_gpu_restarts_match_oracle(gpu_lib):
    """FP64 mirror mode with fixed inner counts, 15^2: three restarts; same sequence of attempts,
    alpha, sweep and iteration counts as the oracle, x to 1e-12.  (Fixed inner counts keep every
    decision of the run far from a tie: the stagnation tests clear the 1% rule by >= 1e-5.)"""
    import torch
    from paper_2512_21164_amd import Solver
    spec, A, x, b, nA = _stagnating_case()
    kw = dict(tol=1e-12, stag_window=5)
    ref = gadi_ref.gadi_select_alpha(A, b, 1e-3, 1.0, spec=spec, normA=nA, max_outer=4000, max_restarts=12,
                                     rule_h=gadi_ref.InnerRule(fixed=6), rule_s=gadi_ref.InnerRule(fixed=3), **kw)
    assert ref.restarts == 3
    s = Solver(gpu_problem(spec), normA=nA, alpha=1e-3, omega=1.0, max_outer=4000, max_restarts=12,
               fixed_inner_h=6, fixed_inner_s=3, **kw)
    bd = to_dev(b)
    xg, rep, hist = s.solve(bd, torch.zeros_like(bd), history=True)
    s.close()
    assert rep["status"] == ref.status == gadi_ref.OK
    assert rep["restarts"] == ref.restarts and rep["alpha"] == pytest.approx(ref.alpha, rel=1e-14)
    assert rep["outer"] == ref.outer and rep["inner_h"] == ref.inner_h and rep["inner_s"] == ref.inner_s
    last = ref.attempts[-1]
    assert rep["attempt_outer"] == last.outer and len(hist) == last.outer + 1
    assert np.max(np.abs(hist[:, 0] - np.array(last.be))) <= 1e-13
    assert rel(xg.cpu().numpy(), ref.x) <= 1e-12


@pytest.mark.gpu
def test_gpu_adaptive_restarts_converge(gpu_lib):
    """Adaptive inner solves: the restarted solve reaches the target where a single attempt stagnates."""
    import torch
    from paper_2512_21164_amd import Solver
    spec, A, x, b, nA = _stagnating_case()
    s = Solver(gpu_problem(spec), normA=nA, alpha=1e-4, omega=1.0, max_outer=3000, max_restarts=12,
               tol=1e-12, stag_window=5)
    bd = to_dev(b)
    xg, rep = s.solve(bd, torch.zeros_like(bd))
    s.close()
    assert rep["status"] == gadi_ref.OK and rep["restarts"] >= 2 and rep["outer"] <= 3000
    assert rep["alpha"] == pytest.approx(1e-4 * G ** rep["restarts"], rel=1e-14)
    assert gadi_ref.backward_error(A, xg.cpu().numpy(), b, nA, extended=True) <= 1.01e-12


@pytest.mark.gpu
def test_gpu_safeguard_raises_alpha_like_oracle(gpu_lib):
    import torch
    from paper_2512_21164_amd import Solver
    spec, A, x, b, nA = _stagnating_case()
    want = gadi_ref.safeguarded_alpha(spec, 1e-3, "bf16", 0.01)
    assert want > 1e-3
    s = Solver(gpu_problem(spec), normA=nA, alpha=1e-3, u_s="bf16", safeguard_tau=0.01, max_outer=3, tol=0.0)
    bd = to_dev(b)
    _, rep = s.solve(bd, torch.zeros_like(bd))
    s.close()
    assert rep["alpha"] == pytest.approx(want, rel=1e-14) and rep["restarts"] == 0
