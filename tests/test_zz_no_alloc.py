"""The allocation-free solve (gadi_solve_noalloc) against the handle-based one (gadi_solve).

Both run the same kernels with the same tile shape on the same inputs, so
every result must be identical: x bitwise, the sweep and inner iteration
counts, the status and the backward-error history.  Three calls in a row
share the library's one static workspace: a 2D 300^2 FP32 solve, a smaller
3D 24^3 BF16 solve (with ||A|| estimated on the device) and the first solve
again, whose result must not depend on what the smaller call left behind.  A
problem larger than the static workspace is refused before any device work.
"""
import numpy as np
import pytest

import workloads
from paper_2512_21164_amd import Problem, Solver, _lib, solve_noalloc, workspace_bytes
from paper_2512_21164_amd.api import make_params

pytestmark = pytest.mark.gpu


def _inputs(pr, seed):
    import torch
    xt = workloads.x_true(pr.size, seed)
    from paper_2512_21164_amd import apply
    return apply(pr, torch.from_numpy(xt).cuda())


def _reference(pr, b, **kw):
    import torch
    s = Solver(pr, **kw)
    x, rep, hist = s.solve(b, torch.zeros_like(b), history=True)
    s.close()
    return x, rep, hist


def _check_same(got, ref):
    (xg, rg, hg), (xr, rr, hr) = got, ref
    assert rg["status"] == rr["status"]
    for k in ("outer", "inner_h", "inner_s", "steps", "attempt_outer"):
        assert rg[k] == rr[k], k
    assert rg["be"] == rr["be"] and rg["normA"] == rr["normA"]
    assert np.array_equal(hg, hr)
    assert np.array_equal(xg.cpu().numpy(), xr.cpu().numpy())


def test_noalloc_matches_handle_solve(gpu_lib):
    import torch
    big = Problem.convection_diffusion(2, 300, 10.0)
    small = Problem.convection_diffusion(3, 24, 5.0)
    kw_big = dict(alpha=0.05, u_s="f32", tol=1e-10, max_outer=4000, normA=8.0)
    kw_small = dict(alpha=0.3, u_s="bf16", tol=1e-10, max_outer=4000)
    assert workspace_bytes(small, make_params(**kw_small)) < workspace_bytes(big, make_params(**kw_big))
    b_big = _inputs(big, 1)
    b_small = _inputs(small, 2)
    ref_big = _reference(big, b_big, **kw_big)
    ref_small = _reference(small, b_small, **kw_small)
    assert ref_big[1]["status"] == 0 and ref_small[1]["status"] == 0
    for pr, b, kw, ref in ((big, b_big, kw_big, ref_big), (small, b_small, kw_small, ref_small),
                           (big, b_big, kw_big, ref_big)):
        x = torch.zeros_like(b)
        got = solve_noalloc(pr, b, x, history=True, **kw)
        print(f"{pr.n} {kw['u_s']}: {got[1]['status_name']} sweeps {got[1]['outer']}", flush=True)
        assert got[0].data_ptr() == x.data_ptr()
        _check_same(got, ref)


def test_noalloc_refuses_problems_beyond_its_workspace(gpu_lib):
    import torch
    pr = Problem.convection_diffusion(2, 2048, 10.0)
    kw = dict(alpha=0.05, u_s="f32", tol=1e-10, max_outer=10, normA=8.0)
    assert workspace_bytes(pr, make_params(**kw)) > _lib.NOALLOC_SCRATCH_BYTES
    b = torch.ones(pr.size, dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 7.0)
    with pytest.raises(_lib.GadiError) as ei:
        solve_noalloc(pr, b, x, **kw)
    assert ei.value.status == _lib.GADI_ERR_CAPACITY
    assert "bytes of device workspace" in str(ei.value)
    assert bool(torch.all(x == 7.0))
