"""Batched execution and the serving loop (GPU).

A member of a batch computes exactly what it computes alone: its tiles, its
reduction order and its state machine do not depend on the other members,
so solutions are compared bitwise.  The serving loop must keep admitted
footprints within the HBM budget, finish every request, and return the same
solutions as solo solves.
"""
import numpy as np
import pytest

import workloads
from oracle import gadi_ref, problems
from tests._problems import gpu_problem, to_dev

pytestmark = pytest.mark.gpu

MIX = [  # (dim, side, beta, alpha, u_s)
    (2, 40, 10.0, 0.3, "f64"),
    (2, 96, 30.0, 0.05, "bf16"),
    (3, 12, 5.0, 0.2, "f64"),
    (2, 33, 0.0, 0.5, "f32"),
    (3, 17, 20.0, 0.1, "bf16"),
    (2, 130, 5.0, 0.02, "f32"),
]


def _case(dim, side, beta, alpha, us, seed):
    import torch
    from paper_2512_21164_amd import Solver
    spec = problems.convection_diffusion(dim, side, (beta,) * dim)
    A = problems.assemble(spec)
    xt = workloads.x_true(spec.size, seed)
    b = A @ xt
    nA = gadi_ref.norm2(A)
    s = Solver(gpu_problem(spec), normA=nA, alpha=alpha, u_s=us, tol=1e-10, max_outer=5000)
    bd = to_dev(b)
    return s, bd, torch.zeros_like(bd), (A, b, nA)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_members_equal_solo_runs(gpu_lib, graph):
    """Five kernel classes in one batch.  On the default stream the steps are launched
    directly; on a created stream they are captured in a graph with one branch per class."""
    import torch
    from paper_2512_21164_amd.batch import Batch
    solo = []
    for i, c in enumerate(MIX):
        s, bd, xd, _ = _case(*c, seed=i)
        x, rep = s.solve(bd, xd)
        solo.append((x.cpu().numpy(), rep))
        s.close()
    stream = torch.cuda.Stream() if graph else None
    batch = Batch(16, stream=stream)
    keep = {}
    for i, c in enumerate(MIX):
        s, bd, xd, sysinfo = _case(*c, seed=i)
        slot = batch.add(s, bd, xd)
        keep[slot] = (i, s, bd, xd, sysinfo)
    reps = batch.run(steps_per_launch=24)
    assert len(reps) == len(MIX)
    for slot, rep in reps.items():
        i, s, bd, xd, (A, b, nA) = keep[slot]
        xs, rs = solo[i]
        assert rep["status"] == 0 and rs["status"] == 0
        assert rep["outer"] == rs["outer"] and rep["inner_h"] == rs["inner_h"] and rep["inner_s"] == rs["inner_s"]
        xb = xd.cpu().numpy()
        assert np.array_equal(xb, xs), MIX[i]
        assert gadi_ref.backward_error(A, xb, b, nA, extended=True) <= 1.01e-10
        s.close()
    batch.close()


def test_batch_many_members_of_one_class(gpu_lib):
    """24 members of one kernel class (2D, FP32 inner solves, sides 130 to 199).  Each
    member's wide tiling has twice the tiles of its inner one, so slots without a tile
    in an inner phase hold a tile of the next outer phase, and 24 descriptors and
    control blocks do not stay in the scalar cache: a slot that read a phase set
    earlier in the same launch would run a tile of the next phase and offset the
    member's ticket counters.  Every member must finish with its solo result."""
    from paper_2512_21164_amd.batch import Batch
    cases = [(2, 130 + 3 * i, 5.0, 0.02, "f32") for i in range(24)]
    batch = Batch(32)
    keep = {}
    for i, c in enumerate(cases):
        s, bd, xd, _ = _case(*c, seed=100 + i)
        keep[batch.add(s, bd, xd)] = (i, s, xd)
    reps = batch.run(steps_per_launch=16)
    assert len(reps) == len(cases)
    for slot, rep in reps.items():
        i, s, xd = keep[slot]
        s2, bd2, xd2, _ = _case(*cases[i], seed=100 + i)
        x2, r2 = s2.solve(bd2, xd2)
        assert rep["status"] == 0 and r2["status"] == 0, cases[i]
        assert (rep["outer"], rep["inner_h"], rep["inner_s"]) == (r2["outer"], r2["inner_h"], r2["inner_s"])
        assert np.array_equal(xd.cpu().numpy(), x2.cpu().numpy()), cases[i]
        s.close()
        s2.close()
    batch.close()


def test_batch_add_while_running(gpu_lib):
    """Members admitted while others are on the device finish with solo results."""
    from paper_2512_21164_amd.batch import Batch
    batch = Batch(8)
    first = [_case(*MIX[i], seed=10 + i) for i in range(3)]
    slots = {batch.add(s, bd, xd): (i, s, bd, xd) for i, (s, bd, xd, _) in enumerate(first)}
    batch.step(40)
    late = [_case(*MIX[i], seed=10 + i) for i in range(3, 6)]
    for j, (s, bd, xd, _) in enumerate(late):
        slots[batch.add(s, bd, xd)] = (3 + j, s, bd, xd)
    reps = batch.run(steps_per_launch=16)
    for slot, rep in reps.items():
        i, s, bd, xd = slots[slot]
        s2, bd2, xd2, _ = _case(*MIX[i], seed=10 + i)
        x2, r2 = s2.solve(bd2, xd2)
        assert np.array_equal(xd.cpu().numpy(), x2.cpu().numpy())
        s.close()
        s2.close()
    batch.close()


def test_serving_loop_budget_and_solo_equality(gpu_lib):
    import torch
    from paper_2512_21164_amd import Solver, apply
    from paper_2512_21164_amd.serve import Server, request_problem, summarize
    trace = workloads.scale_trace(workloads.poisson_trace(num=20, rate_per_s=400.0, seed=3), 80, 20)
    trace = [t for t in trace]
    srv = Server(budget_bytes=0, max_slots=8, u_s="bf16", max_outer=3000, keep_solutions=True)
    fps = [srv.footprint(r) for r in trace]
    srv.budget = int(2.5 * max(fps))          # admission binds: only a few fit at once
    res = srv.run(trace)
    summ = summarize(res)
    assert summ["completed"] == len(trace)
    assert srv.max_used <= srv.budget
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0
    for r in res[:5]:
        req = next(q for q in trace if q.rid == r.rid)
        pr = request_problem(req)
        xt = torch.from_numpy(workloads.x_true(pr.size, req.seed)).cuda()
        b = apply(pr, xt)
        s = Solver(pr, alpha=req.alpha, u_s="bf16", tol=1e-10, max_outer=3000, norm_iters=30,
                   tile_chunk=srv.params.get("tile_chunk", 0))      # the server's tiling of its members
        x, rep = s.solve(b, torch.zeros_like(b))
        s.close()
        assert rep["status_name"] == r.status
        assert np.array_equal(x.cpu().numpy(), srv.solutions[r.rid])
    srv.close()


def test_serving_with_predicted_alpha(gpu_lib):
    """alpha_source="gpr": each request starts from the packaged model's alpha (Section 4.2);
    the served result equals a solo solve with that alpha, bit for bit."""
    import torch
    from paper_2512_21164_amd import Solver, apply
    from paper_2512_21164_amd.alpha_gpr import Model
    from paper_2512_21164_amd.serve import Server, request_problem, summarize
    trace = workloads.scale_trace(workloads.poisson_trace(num=8, rate_per_s=400.0, seed=5), 96, 24)
    srv = Server(budget_bytes=1 << 30, max_slots=4, u_s="f32", max_outer=3000, keep_solutions=True,
                 alpha_source="gpr")
    res = srv.run(trace)
    summ = summarize(res)
    assert summ["completed"] == len(trace)
    model = Model.load()
    for r in res[:4]:
        req = next(q for q in trace if q.rid == r.rid)
        pr = request_problem(req)
        a = model.predict(pr, "f32")[0]
        assert srv.alpha(req) == a
        xt = torch.from_numpy(workloads.x_true(pr.size, req.seed)).cuda()
        b = apply(pr, xt)
        s = Solver(pr, alpha=a, u_s="f32", tol=1e-10, max_outer=3000, norm_iters=30,
                   tile_chunk=srv.params.get("tile_chunk", 0))
        x, rep = s.solve(b, torch.zeros_like(b))
        s.close()
        assert rep["status_name"] == r.status
        assert np.array_equal(x.cpu().numpy(), srv.solutions[r.rid])
    model.close()
    srv.close()


def test_serving_stall_watchdog_raises(gpu_lib):
    """Failure detection, forced from the host: with a zero stall limit the loop raises as soon
    as a step passes without a request finishing; the device stays usable."""
    import torch
    from paper_2512_21164_amd import Solver, apply
    from paper_2512_21164_amd.serve import Server, request_problem
    trace = workloads.scale_trace(workloads.poisson_trace(num=4, rate_per_s=1000.0, seed=7), 64, 16)
    srv = Server(budget_bytes=1 << 30, max_slots=4, u_s="f32", max_outer=3000, stall_timeout_s=0.0)
    with pytest.raises(RuntimeError, match="stalled"):
        srv.run(trace)
    torch.cuda.synchronize()
    srv.close()
    pr = request_problem(trace[0])
    xt = torch.from_numpy(workloads.x_true(pr.size, 0)).cuda()
    b = apply(pr, xt)
    s = Solver(pr, alpha=trace[0].alpha, u_s="f32", tol=1e-8, max_outer=3000)
    _, rep = s.solve(b, torch.zeros_like(b))
    s.close()
    assert rep["status"] in (0, 1, 2, 3)
