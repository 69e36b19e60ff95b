#!/usr/bin/env python3
"""Benchmark of mixed-precision GADI on one MI355X.

A step is one complete GADI solve (Algorithm 1 of arXiv 2512.21164) of a
synthetic system to backward error 1e-10, inputs resident in HBM: the mixed
precision solve (FP64 residual, update and norms; inner CG / CGNE in BF16
storage with FP32 arithmetic, or FP32) is timed, and the same solve with FP64
inner solves is timed beside it.

Default workload: 2D convection-diffusion, 4096 x 4096 interior grid
(1.68e7 unknowns), 5-point stencil, convection (10, 10), omega = 1,
x_true ~ U(-1, 1) seed 0, b = A x_true formed on the device; alpha = 7.197e-3
(the third of eight log-spaced values of [1e-3, 1]) and inner tolerance 1e-2
(from the paper's set 1e-2 .. 1e-6), the fastest pair of the parameter study
for both precisions.

Prints ONE JSON line (value = mixed-precision solves per second) with a
roofline object for the step kernel (algorithmic bytes per launch over the
event-timed average launch duration) and a cpu_baseline object (the CPU
oracle on a bounded sample, extrapolated).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    # name: (dim, ng, beta, default alpha, description)
    "c2": (2, 4096, 10.0, 7.1969e-3, "2D convection-diffusion 4096x4096 (1.68e7 unknowns), 5-point stencil"),
    "c3": (3, 512, 10.0, 5.179e-2, "3D convection-diffusion 512^3 (1.34e8 unknowns), 7-point stencil"),
    "c1": (2, 64, 1.0, 0.5, "2D convection-diffusion 64x64 (4096 unknowns), 5-point stencil"),
}
SBYTES = {"f64": 8, "f32": 4, "bf16": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--us", default="f32", choices=["bf16", "f32"], help="inner precision of the mixed solve")
    ap.add_argument("--u-r", default="f64", choices=["f64", "f64x2"],
                    help="residual precision u_r: FP64, or FP64 pairs (extra precision) for both solves")
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--alpha", default=None,
                    help="regularization alpha (a number), or 'gpr' for the packaged Section 4.2 model")
    ap.add_argument("--max-restarts", type=int, default=0,
                    help="alpha restarts on stagnation or divergence (Section 4.3, step 3)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--inner-tol", type=float, default=1e-2,
                    help="relative-residual tolerance of both inner solves (the paper picks it from 1e-2..1e-6)")
    ap.add_argument("--max-outer", type=int, default=20000)
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed FP64-inner solves (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=1, help="oracle sweeps timed for the CPU baseline")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3)")
    return ap.parse_args()


def alg_bytes(hist, n, s, w=8, cplx=False):
    """Algorithmic HBM bytes of one solve from its per-sweep iteration counts.

    Per unknown (s = bytes of a u_s element, w = bytes of an FP64 element):
    IMPORT 4w; OUTER k=0: 2w+s, k>=1: 3w+3s (3w+2s when the last inner solve
    took one iteration); CG(H): first pass 2s / 4s / 5s for j = 0 / 1 / >=2,
    second pass 3s; CGNE(S): start 4s (3s when CG took one iteration), first
    pass 4s / 5s for j = 1 / >=2, second pass 3s; EXPORT 2w.
    """
    if cplx:
        w, s = 2 * w, 2 * s
    total = 4 * w
    K = len(hist) - 1
    for k in range(K + 1):
        if k == 0:
            total += 2 * w + s
        else:
            prev_last = int(hist[k - 1][2] if cplx else hist[k - 1][3])
            total += 3 * w + (3 * s if prev_last >= 2 else 2 * s)
        if k == K:
            break
        jh, js = int(hist[k][2]), int(hist[k][3])
        for j in range(jh):
            total += (2 * s if j == 0 else 4 * s if j == 1 else 5 * s) + 3 * s
        if not cplx and js > 0:
            total += 4 * s if jh >= 2 else 3 * s
            for j in range(js):
                total += 3 * s + (0 if j == 0 else (4 * s if j == 1 else 5 * s))
    total += 2 * w
    return float(total) * n


def kernel_sources_sha256():
    """Hash of the sources of the step kernel and of its launch configuration (tilings,
    grid, chunking): the traffic record is valid only for these."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2512_21164_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "gadi_step*")))
    files += [os.path.join(csrc, f) for f in ("gadi_kernels.hip", "gadi_internal.h", "gadi_launch.h", "gadi_api.cpp")]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, us, alpha, beta, inner_tol, u_r="f64"):
    """HBM bytes per step launch from the committed rocprofv3 counter runs, or None.

    The record (profiles/gadi_step_<us>_2d4096_traffic.json) holds FETCH_SIZE + WRITE_SIZE per
    launch, each scaled by the same counter's reading on a plain 1 GiB copy; it is used only
    for the workload it was taken on and only while the kernel sources are unchanged.
    """
    path = os.path.join(ROOT, "profiles", f"gadi_step_{us}_2d4096_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    same = (rec.get("workload") == workload and rec.get("u_s") == us and abs(rec.get("alpha", -1) - alpha) < 1e-12
            and abs(rec.get("beta", -1) - beta) < 1e-12 and abs(rec.get("inner_tol", -1) - inner_tol) < 1e-15
            and rec.get("u_r", "f64") == u_r
            and rec.get("source_sha256") == kernel_sources_sha256())
    return float(rec["traffic_bytes_per_launch"]) if same else None


def cpu_baseline(dim, ng, beta, alpha, x_true_np, mh, ms, sweeps, us, gpu_outer, normA):
    """Oracle (CPU, FP64 / emulated u_s) time per sweep on this workload, extrapolated."""
    from threadpoolctl import threadpool_limits
    from oracle import gadi_ref, problems
    with threadpool_limits(1):
        spec = problems.convection_diffusion(dim, ng, (beta,) * dim)
        A = problems.assemble(spec)
        b = A @ x_true_np
        rh = gadi_ref.InnerRule(fixed=max(1, mh))
        rs = gadi_ref.InnerRule(fixed=max(1, ms))
        t0 = time.perf_counter()
        gadi_ref.gadi(A, b, alpha, 1.0, normA=normA, max_outer=0, tol=0.0, prec=us, rule_h=rh, rule_s=rs)
        t1 = time.perf_counter()
        gadi_ref.gadi(A, b, alpha, 1.0, normA=normA, max_outer=sweeps, tol=0.0, prec=us, rule_h=rh, rule_s=rs,
                      stag_window=0, div_factor=0.0)
        t2 = time.perf_counter()
    per_sweep = max((t2 - t1) - (t1 - t0), 1e-9) / sweeps
    solve_s = per_sweep * gpu_outer
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"{sweeps} GADI sweep(s) of this workload in the NumPy/SciPy oracle "
                       f"(u_s={us} emulated, CG {mh} + CGNE {ms} iterations per sweep = the GPU's mean), "
                       f"{per_sweep:.2f} s/sweep single-threaded, extrapolated to the GPU's {gpu_outer} sweeps "
                       f"({solve_s:.1f} s per solve)")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    from paper_2512_21164_amd import Problem, Solver, apply

    dim, ng, beta0, alpha0, desc = WORKLOADS[args.workload]
    beta = beta0 if args.beta is None else args.beta
    pr = Problem.convection_diffusion(dim, ng, beta)
    alpha_source = "fixed"
    if args.alpha is None:
        alpha = alpha0
    elif args.alpha == "gpr":
        from paper_2512_21164_amd.alpha_gpr import predict_alpha
        alpha = predict_alpha(pr, args.us)
        alpha_source = "gpr"
    else:
        alpha = float(args.alpha)
    n = pr.size
    dev = torch.device("cuda:0")
    x_np = workloads.x_true(n, 0, "normal" if dim == 3 else "uniform")
    xt = torch.from_numpy(x_np).to(dev)
    b = apply(pr, xt)
    torch.cuda.synchronize()
    nxt = torch.linalg.norm(xt)

    def run(us, steps, warmup):
        s = Solver(pr, alpha=alpha, omega=1.0, u_s=us, u_r=args.u_r, tol=args.tol, max_outer=args.max_outer,
                   inner_tol_h=args.inner_tol, inner_tol_s=args.inner_tol, max_restarts=args.max_restarts)
        reps = []
        x = torch.zeros_like(b)
        for _ in range(warmup):
            x.zero_()
            _, wrep = s.solve(b, x)
            print(f"[bench] {us} warm-up solve: {wrep['status_name']} outer={wrep['outer']} ms={wrep['ms']:.1f}",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            x.zero_()
            x, rep, hist = s.solve(b, x, history=True)
            reps.append((rep, hist))
            print(f"[bench] {us} solve {i + 1}/{steps}: {rep['status_name']} outer={rep['outer']} "
                  f"inner_h={rep['inner_h']} inner_s={rep['inner_s']} be={rep['be']:.3e} ms={rep['ms']:.1f}",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        fe = float(torch.linalg.norm(x - xt) / nxt)
        normA = s.normA
        s.close()
        return el, reps, fe, normA

    el, reps, fe, normA = run(args.us, args.steps, args.warmup)
    rep, hist = reps[-1]
    value = args.steps / el
    s_b = SBYTES[args.us]
    bytes_solve = alg_bytes(hist, n, s_b)
    kern_ms = float(np.mean([r["kernel_ms"] for r, _ in reps]))
    launches = float(np.mean([r["steps"] for r, _ in reps]))
    avg_launch_us = 1000.0 * kern_ms / launches
    achieved = (bytes_solve / launches) / (avg_launch_us * 1e-6) / 1e9

    out = {
        "metric": "time-to-1e-10 backward error & solves/s, mixed vs FP64 GADI; HBM GB/s",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"f64+{args.us}", "data": "synthetic",
        "config": {"workload": f"{desc}, beta=({beta},{beta}{',' + str(beta) if dim == 3 else ''}), "
                               f"alpha={alpha}, omega=1, inner tolerance {args.inner_tol}, target backward error {args.tol}"
                               + (", residual in FP64 pairs" if args.u_r == "f64x2" else ""),
                   "grid": [ng] * dim, "unknowns": n, "inner_precision": args.us, "alpha": alpha, "beta": beta,
                   "inner_tol": args.inner_tol, "residual_precision": args.u_r, "alpha_source": alpha_source,
                   "max_restarts": args.max_restarts},
        "time_to_solution_s": el / args.steps,
        "mixed": {"u_s": args.us, "status": rep["status_name"], "outer": rep["outer"], "inner_h": rep["inner_h"],
                  "inner_s": rep["inner_s"], "be": rep["be"], "forward_error": fe, "solve_ms": rep["ms"],
                  "kernel_ms": rep["kernel_ms"], "launches": rep["steps"], "alg_bytes_per_solve": bytes_solve,
                  "alpha_final": rep["alpha"], "restarts": rep["restarts"]},
    }
    if args.fp64_steps > 0:
        el64, reps64, fe64, _ = run("f64", args.fp64_steps, 0)
        r64, h64 = reps64[-1]
        out["fp64"] = {"solves_per_s": args.fp64_steps / el64, "time_to_solution_s": el64 / args.fp64_steps,
                       "status": r64["status_name"], "outer": r64["outer"], "inner_h": r64["inner_h"],
                       "inner_s": r64["inner_s"], "be": r64["be"], "forward_error": fe64,
                       "alg_bytes_per_solve": alg_bytes(h64, n, 8)}
        out["speedup_mixed_vs_fp64"] = value / out["fp64"]["solves_per_s"]
    kname = {"bf16": "gadi::gadi_step<gadi::bf16, %d, %d, %s>", "f32": "gadi::gadi_step<float, %d, %d, %s>"}[args.us]
    if any(r["restarts"] > 0 for r, _ in reps):
        # the sweep history holds the last attempt only: the bytes of a restarted solve are not known
        achieved = None
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
                       "traffic": measured_traffic(args.workload, args.us, alpha, beta, args.inner_tol, args.u_r),
                       "kernel": kname % (dim, 1, "true" if args.u_r == "f64x2" else "false"),
                       "avg_launch_us": avg_launch_us, "alg_bytes_per_launch": bytes_solve / launches}
    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu:
        print("[bench] CPU oracle baseline (bounded sample) ...", file=sys.stderr, flush=True)
        mh = int(round(rep["inner_h"] / max(1, rep["outer"])))
        ms = int(round(rep["inner_s"] / max(1, rep["outer"])))
        out["cpu_baseline"] = cpu_baseline(dim, ng, beta, alpha, x_np, mh, ms, args.cpu_sweeps, args.us,
                                           int(rep["outer"]), normA)
        if args.u_r != "f64":
            out["cpu_baseline"]["sample"] += "; the oracle forms the residual in FP64 (its exact residual is not timed)"
        print("[bench] CPU oracle baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
