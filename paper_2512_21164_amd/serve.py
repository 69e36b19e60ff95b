"""Continuous-batching request loop for GADI solves on one GPU.

Requests (a convection-diffusion system each) arrive over time.  The loop
admits a waiting request when a batch slot is free and its HBM footprint
(workspace + b + x) fits in the remaining budget, creates its solver on a
side stream while the batch stream runs the step enqueued just before (so
the norm estimate and right-hand side overlap the running batch), and adds it
to the batch, whose members keep their Krylov state resident until they
finish.  After each step the batch is polled (one gather of all members'
control blocks), finished members are retired and their memory is released.  The loop reports per-request latency
(arrival to result), p50 / p99, and solves per second over the makespan.

Each request carries its own alpha; with ``alpha_source="gpr"`` the server
instead starts every request from the alpha that the packaged regression
model predicts for it (Section 4.2; the model was trained with FP32 and BF16
inner solves, so FP64 inner solves take the FP32 prediction, where the
kappa(H) kappa(S) u_s term is already negligible).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List

import numpy as np

from .api import Problem, Solver, apply, make_params, workspace_bytes
from .batch import Batch


@dataclasses.dataclass
class Result:
    rid: int
    arrival_s: float
    admitted_s: float
    finished_s: float
    status: str
    outer: int
    inner_h: int
    inner_s: int
    be: float
    forward_error: float
    n: int
    footprint: int

    @property
    def latency_s(self) -> float:
        return self.finished_s - self.arrival_s


def request_problem(req) -> Problem:
    return Problem.convection_diffusion(req.dim, req.side, req.beta)


class Server:
    """Admission by HBM footprint + continuous batching over the C-ABI batch."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, u_s: str = "f64", tol: float = 1e-10,
                 max_outer: int = 20000, norm_iters: int = 30, steps_per_launch: int = 16, device="cuda",
                 keep_solutions: bool = False, alpha_source: str = "request", stall_timeout_s=None,
                 autotune: bool = False, client_payload: bool = False, tile_share: int = 4):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.params = dict(u_s=u_s, tol=tol, max_outer=max_outer, norm_iters=norm_iters, omega=1.0)
        # tile_share k > 1: each request is tiled with k times fewer (longer) tiles than a system
        # that has the device to itself, since it shares every batch launch with the other members
        # (every tile of a launch pays a reduction and a ticket; on the serving trace k = 4 served
        # 27% more FP32 solves per second than k = 1, and k = 2, 6, 8, 16 less than k = 4)
        if tile_share > 1:
            self.params["tile_chunk"] = -int(tile_share)
        self.U = int(steps_per_launch)
        self.stream = torch.cuda.Stream(device=self.device)
        self.side = torch.cuda.Stream(device=self.device)
        self.batch = Batch(self.max_slots, stream=self.stream, device=self.device)
        self.keep = keep_solutions
        self.solutions: Dict[int, np.ndarray] = {}
        self.max_used = 0
        if alpha_source not in ("request", "gpr"):
            raise ValueError("alpha_source must be 'request' or 'gpr'")
        self.model = None
        if alpha_source == "gpr":
            from .alpha_gpr import Model
            self.model = Model.load()
        self._alpha_cache: Dict[int, float] = {}
        # failure detection: with requests on the device, at least one must finish
        # within this many seconds, else run() raises (None: no limit)
        self.stall_timeout_s = stall_timeout_s
        # tile shapes: with autotune, the first request of each kernel and size class has the
        # library time the candidate shapes (once per class and process); every later handle of
        # the class uses the choice
        self.autotune = bool(autotune)
        # client_payload: each request brings its right-hand side's data with it (generated, as a client
        # would, before the trace starts, and kept in pinned host memory); otherwise the loop draws
        # x_true at admission
        self.client_payload = bool(client_payload)
        self._payload: Dict[int, object] = {}
        # host seconds per part of the loop (admission, step enqueue, poll, retire, add)
        self.host_s = collections.Counter()

    def alpha(self, req) -> float:
        """The request's alpha, or the model's prediction for its problem."""
        if self.model is None:
            return req.alpha
        if req.rid not in self._alpha_cache:
            us = self.params["u_s"]
            self._alpha_cache[req.rid] = self.model.predict(request_problem(req), "f32" if us == "f64" else us)[0]
        return self._alpha_cache[req.rid]

    def footprint(self, req) -> int:
        pr = request_problem(req)
        p = make_params(alpha=self.alpha(req), **self.params)
        return workspace_bytes(pr, p) + 3 * 8 * pr.size     # workspace + b, x, x_true

    def _start(self, req):
        import workloads
        torch = self.torch
        pr = request_problem(req)
        with torch.cuda.stream(self.side):
            if req.rid in self._payload:
                xt = self._payload.pop(req.rid).to(self.device, non_blocking=True)
            else:
                xt = torch.from_numpy(workloads.x_true(pr.size, req.seed)).to(self.device, non_blocking=False)
            b = apply(pr, xt, stream=self.side)
            x = torch.zeros_like(b)
            s = Solver(pr, stream=self.side, device=self.device, alpha=self.alpha(req), autotune=self.autotune,
                       **self.params)
        self.side.synchronize()
        return s, b, x, xt

    def run(self, trace, time_scale: float = 1.0, log=None) -> List[Result]:
        """Serve the requests of ``trace`` (arrival times scaled by time_scale).

        Each round enqueues the next batch step first, then prepares newly admitted
        requests (right-hand side, solver set-up and norm estimate) on the side stream
        while the device runs that step, then polls the batch, retires finished members
        and adds the prepared requests."""
        torch = self.torch
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival_s))
        waiting = collections.deque()
        active = {}
        used = 0
        results: List[Result] = []
        if self.client_payload:
            import workloads
            for req in trace:
                self._payload[req.rid] = torch.from_numpy(workloads.x_true(req.side ** req.dim, req.seed)).pin_memory()
        hs = self.host_s
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        last_progress = 0.0
        while pending or waiting or active:
            t = now()
            while pending and pending[0].arrival_s * time_scale <= t:
                waiting.append(pending.popleft())
            stepped = bool(active)
            tq = time.perf_counter()
            if stepped:
                self.batch.step(self.U)          # asynchronous: the device runs it during admission
            ta = time.perf_counter()
            hs["step"] += ta - tq
            prepared = []
            while waiting and len(active) + len(prepared) < self.max_slots:
                req = waiting[0]
                fp = self.footprint(req)
                if fp > self.budget:
                    waiting.popleft()
                    results.append(Result(req.rid, req.arrival_s * time_scale, now(), now(), "REJECTED", 0, 0, 0,
                                          float("nan"), float("nan"), req.n, fp))
                    continue
                if used + fp > self.budget:
                    break
                waiting.popleft()
                t_adm = now()
                t1 = time.perf_counter()
                s, b, x, xt = self._start(req)
                hs["admit"] += time.perf_counter() - t1
                hs["admitted"] += 1
                prepared.append((req, t_adm, fp, s, b, x, xt))
                used += fp
                self.max_used = max(self.max_used, used)
            if stepped:
                tp = time.perf_counter()
                done, _ = self.batch.poll()
                tr = time.perf_counter()
                hs["poll"] += tr - tp
                hs["rounds"] += 1
                for slot in done:
                    s, b, x, rep = self.batch.remove(slot)
                    req, t_adm, fp, xt = active.pop(slot)
                    fe = float(torch.linalg.norm(x - xt) / torch.linalg.norm(xt))
                    if self.keep:
                        self.solutions[req.rid] = x.cpu().numpy()
                    results.append(Result(req.rid, req.arrival_s * time_scale, t_adm, now(), rep["status_name"],
                                          rep["outer"], rep["inner_h"], rep["inner_s"], rep["be"], fe, req.n, fp))
                    s.close()
                    del s, b, x, xt
                    used -= fp
                    last_progress = now()
                    if log:
                        log(results[-1])
                hs["retire"] += time.perf_counter() - tr
            tb = time.perf_counter()
            for req, t_adm, fp, s, b, x, xt in prepared:
                slot = self.batch.add(s, b, x)
                active[slot] = (req, t_adm, fp, xt)
                last_progress = now()
            hs["add"] += time.perf_counter() - tb
            if active and self.stall_timeout_s is not None and now() - last_progress > self.stall_timeout_s:
                stuck = sorted(req.rid for req, _, _, _ in active.values())
                raise RuntimeError(f"serving stalled: no request finished or was admitted for "
                                   f"{now() - last_progress:.1f} s; active requests {stuck}")
            if not active and not prepared and pending:
                time.sleep(max(0.0, min(0.002, pending[0].arrival_s * time_scale - now())))
        return results

    def close(self):
        self.batch.close()
        if self.model is not None:
            self.model.close()


def summarize(results: List[Result]) -> dict:
    done = [r for r in results if r.status != "REJECTED"]
    lat = np.array([r.latency_s for r in done]) if done else np.array([np.nan])
    first = min(r.arrival_s for r in results)
    last = max(r.finished_s for r in results)
    return {
        "requests": len(results),
        "completed": len(done),
        "converged": sum(r.status == "OK" for r in done),
        "not_converged": sum(r.status != "OK" for r in done),
        "rejected": sum(r.status == "REJECTED" for r in results),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(np.mean(lat)),
        "makespan_s": last - first,
        "solves_per_s": len(done) / max(last - first, 1e-9),
        "max_backward_error_converged": float(max([r.be for r in done if r.status == "OK"], default=np.nan)),
    }


__all__ = ["Server", "Result", "summarize", "request_problem"]


def main(argv=None):
    """Serve a Poisson trace of convection-diffusion requests; print a JSON summary per precision."""
    import argparse
    import json
    import sys

    import workloads
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-side2d", type=int, default=1024)
    ap.add_argument("--max-side3d", type=int, default=128)
    ap.add_argument("--budget-gb", type=float, default=2.0, help="HBM admission budget")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--max-outer", type=int, default=20000)
    ap.add_argument("--steps-per-launch", type=int, default=16)
    ap.add_argument("--us", default="bf16,f64", help="comma-separated inner precisions to run, in order")
    ap.add_argument("--alpha", default="request", choices=["request", "gpr"],
                    help="alpha of each solve: the request's, or the packaged model's prediction")
    ap.add_argument("--autotune", action="store_true", help="tune the tile shape of each request class on first use")
    ap.add_argument("--tile-share", type=int, default=4,
                    help="tile each request with k times fewer tiles than a system alone on the device")
    ap.add_argument("--client-payload", action="store_true",
                    help="requests bring their data (x_true drawn before the trace starts, pinned host memory)")
    ap.add_argument("--results", default=None,
                    help="write one JSON line per request (per precision) to this file")
    ap.add_argument("--stall-timeout", type=float, default=600.0,
                    help="raise if no request finishes or is admitted for this many seconds (0: off)")
    args = ap.parse_args(argv)
    trace = workloads.scale_trace(workloads.poisson_trace(args.requests, args.rate, args.seed),
                                  args.max_side2d, args.max_side3d)
    out = {}
    for us in args.us.split(","):
        srv = Server(int(args.budget_gb * 2 ** 30), max_slots=args.slots, u_s=us, max_outer=args.max_outer,
                     steps_per_launch=args.steps_per_launch, alpha_source=args.alpha,
                     stall_timeout_s=args.stall_timeout if args.stall_timeout > 0 else None, autotune=args.autotune,
                     client_payload=args.client_payload, tile_share=args.tile_share)
        done = [0]

        def log(r, us=us):
            done[0] += 1
            if done[0] % 16 == 0 or done[0] == len(trace):
                print(f"[serve {us}] {done[0]}/{len(trace)} done, last: rid={r.rid} n={r.n} {r.status} "
                      f"outer={r.outer} latency={r.latency_s:.3f}s", file=sys.stderr, flush=True)
        res = srv.run(trace, log=log)
        if args.results:
            by_id = {r.rid: r for r in trace}
            with open(args.results, "a") as fh:
                for r in res:
                    q = by_id[r.rid]
                    fh.write(json.dumps({"u_s": us, "rid": r.rid, "dim": q.dim, "side": q.side, "n": r.n,
                                         "beta": q.beta, "arrival_s": r.arrival_s, "admitted_s": r.admitted_s,
                                         "finished_s": r.finished_s, "status": r.status, "outer": r.outer,
                                         "inner_h": r.inner_h, "inner_s": r.inner_s, "be": r.be,
                                         "footprint": r.footprint}) + "\n")
        summ = summarize(res)
        summ["host_s"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in srv.host_s.items()}
        summ["max_admitted_bytes"] = srv.max_used
        summ["budget_bytes"] = srv.budget
        out[us] = summ
        srv.close()
    print(json.dumps({"serving": out, "requests": args.requests, "rate_per_s": args.rate,
                      "max_side2d": args.max_side2d, "max_side3d": args.max_side3d, "max_outer": args.max_outer,
                      "alpha": args.alpha, "autotune": args.autotune, "client_payload": args.client_payload,
                      "steps_per_launch": args.steps_per_launch, "tile_share": args.tile_share}))


if __name__ == "__main__":
    main()
