#!/usr/bin/env python3
"""Benchmark of mixed-precision GADI on one MI355X.

A step is one complete GADI solve (Algorithm 1 of arXiv 2512.21164) of a
synthetic system to backward error 1e-10, inputs resident in HBM: the mixed
precision solve (FP64 residual, update and norms; inner CG / CGNE in FP32, or
BF16 storage with FP32 arithmetic) is timed, and the same solve with FP64
inner solves is timed beside it.

Default workload: 3D convection-diffusion, 512^3 interior grid (1.34e8
unknowns), 7-point stencil, convection (10, 10, 10), omega = 1, x_true ~
N(0, 1) seed 0, b = A x_true formed on the device, FP32 inner solves;
alpha from the packaged Gaussian-process model (the data-driven initial alpha of
Section 4.2: 1.756e-2 for this problem, close to the fastest alpha of a scan) and
inner tolerance 1e-2 (from the paper's set 1e-2 .. 1e-6, the fastest here).  The 2D 4096^2 workload (--workload c2) remains
available.

Prints ONE JSON line (value = mixed-precision solves per second) with a
roofline object for the step kernel and a cpu_baseline object (the CPU
oracle on a bounded sample, extrapolated).  Algorithmic bytes of the roofline
are the per-unit figures of the method: an outer sweep moves 24 + 2s bytes per
unknown (x, b read and x written in FP64, the residual written in u_s with s
bytes per element) and a CG or CGNE iteration 10s (four vector reads and
writes plus the stored product q); complex problems double both.  This
implementation recomputes q instead of storing it and moves fewer bytes
(``alg_bytes_design``); both rates are reported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    # name: (dim, ng, beta, default alpha ("gpr": the packaged regression model's prediction),
    #        default inner tolerance, description, oracle sample grid side)
    "c3": (3, 512, 10.0, "gpr", 1e-2, "3D convection-diffusion 512^3 (1.34e8 unknowns), 7-point stencil", 128),
    "c2": (2, 4096, 10.0, 7.1969e-3, 1e-2, "2D convection-diffusion 4096x4096 (1.68e7 unknowns), 5-point stencil",
           4096),
    "c1": (2, 64, 1.0, 0.5, 1e-3, "2D convection-diffusion 64x64 (4096 unknowns), 5-point stencil", 64),
}
# profiles/ file tag of each workload's counter record
TRAFFIC_TAG = {"c3": "3d512", "c2": "2d4096", "c1": "2d64"}
SBYTES = {"f64": 8, "f32": 4, "bf16": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--us", default="f32", choices=["bf16", "f32", "f64"],
                    help="inner precision of the timed solve (f64: plain FP64 GADI, for profiles)")
    ap.add_argument("--u-r", default="f64", choices=["f64", "f64x2"],
                    help="residual precision u_r: FP64, or FP64 pairs (extra precision) for both solves")
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--alpha", default=None,
                    help="regularization alpha (a number), or 'gpr' for the packaged Section 4.2 model")
    ap.add_argument("--max-restarts", type=int, default=0,
                    help="alpha restarts on stagnation or divergence (Section 4.3, step 3)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="relative-residual tolerance of both inner solves (the paper picks it from 1e-2..1e-6); "
                         "default: the workload's (1e-2)")
    ap.add_argument("--max-outer", type=int, default=20000)
    ap.add_argument("--fixed-inner", default=None,
                    help="H,S: run exactly H CG and S CGNE iterations per sweep (with --tol 0 and --max-outer K a "
                         "fixed phase sequence, for per-phase profiles)")
    ap.add_argument("--normA", type=float, default=0.0, help="||A||_2 to use (0: estimate on the device)")
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed FP64-inner solves (0: skip)")
    ap.add_argument("--fp64-warmup", type=int, default=1, help="untimed FP64-inner solves before the timed ones")
    ap.add_argument("--bf16-steps", type=int, default=1,
                    help="timed solves with BF16-stored inner vectors beside the FP32 ones (0: skip)")
    ap.add_argument("--bf16-warmup", type=int, default=1)
    ap.add_argument("--tile-ry", type=int, default=0, help="3D rows per wave (0: library default)")
    ap.add_argument("--tile-chunk", type=int, default=0,
                    help="planes per wave tile of the inner phases (0: library default; -k: k times the default)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate tile shapes first (gadi_autotune) and solve with the fastest")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=0,
                    help="oracle sweeps timed for the CPU baseline (0: as many as fill --cpu-seconds)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU time the oracle sample is sized for when --cpu-sweeps is 0")
    ap.add_argument("--cpu-grid", type=int, default=0,
                    help="grid side of the oracle's sample (0: the workload's; below the full side the "
                         "time is scaled by the unknown count)")
    ap.add_argument("--no-calib", action="store_true", help="skip the HBM stream calibration")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3)")
    return ap.parse_args()


def alg_bytes(hist, n, s, w=8, cplx=False, pair_z=None, dim=3, ry=1):
    """Bytes this implementation must move in one solve, from its per-sweep iteration counts.

    Per unknown (s = bytes of a u_s element, w = bytes of an FP64 element):
    IMPORT 4w; OUTER k=0: 2w+s, k>=1: 3w+3s (3w+2s when the last inner solve
    took one iteration); CG(H) with z updated every second iteration (FP32
    and FP64 real problems, complex128, complex64 in 2D, real BF16 in 3D with ry >= 2 rows per
    wave: pair_z): first pass 2s / 3s for j = 0 / odd j,
    5s / 6s for j = 2 / even j >= 4, and after an even count J the z fold (2s
    for J = 2, else 3s); without pairing: first pass 2s / 4s / 5s for
    j = 0 / 1 / >= 2; second pass 3s;
    CGNE(S): start 4s (3s when CG took one iteration), first pass 4s / 5s for
    j = 1 / >=2, second pass 3s; EXPORT 2w.
    """
    if pair_z is None:
        pair_z = (s >= 4 and (not cplx or s == 8 or dim == 2)) or (s == 2 and not cplx and dim == 3 and ry >= 2)
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
            if pair_z:
                first = 2 * s if j == 0 else (3 * s if j % 2 else (5 * s if j == 2 else 6 * s))
            else:
                first = 2 * s if j == 0 else (4 * s if j == 1 else 5 * s)
            total += first + 3 * s
        if pair_z and jh >= 2 and jh % 2 == 0:
            total += 2 * s if jh == 2 else 3 * s
        if not cplx and js > 0:
            total += 4 * s if jh >= 2 else 3 * s
            for j in range(js):
                total += 3 * s + (0 if j == 0 else (4 * s if j == 1 else 5 * s))
    total += 2 * w
    return float(total) * n


def alg_bytes_unit(outer, inner_h, inner_s, n, s, cplx=False):
    """Algorithmic bytes of one solve from the method's per-unit figures.

    Per unknown: an outer sweep 24 + 2s (x and b read, x written in FP64, the
    residual written in u_s and read back by the first inner pass), a CG
    iteration on H or a CGNE iteration on S 10s (p, r, z / y and q = H p or
    S p read or written once each); complex elements double both.
    """
    f = 2 if cplx else 1
    return float(n) * f * ((24 + 2 * s) * outer + 10 * s * (inner_h + inner_s))


def kernel_sources_sha256():
    """Hash of the device sources of the step kernel; with the tile shape recorded beside it
    (rows per wave, chunk lengths, tiles) it identifies the launches a traffic record covers."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2512_21164_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "gadi_step*")))
    files += [os.path.join(csrc, f) for f in ("gadi_kernels.hip", "gadi_internal.h", "gadi_launch.h")]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record(workload, us, alpha, beta, inner_tol, u_r="f64", tiling=None):
    """The committed rocprofv3 counter record of this workload and step kernel, or None.

    The record (profiles/gadi_step_<us>_<workload tag>_traffic.json) holds FETCH_SIZE + WRITE_SIZE
    over the step launches of a truncated solve of the workload, each counter scaled by its reading
    on a plain 1 GiB copy, and their ratio to the bytes this implementation must move over the same
    launches.  It is used only for the workload and tile shape it was taken on and only while the
    kernel sources are unchanged.
    """
    path = os.path.join(ROOT, "profiles", f"gadi_step_{us}_{TRAFFIC_TAG.get(workload, workload)}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    same = (rec.get("workload") == workload and rec.get("u_s") == us and abs(rec.get("alpha", -1) - alpha) < 1e-12
            and abs(rec.get("beta", -1) - beta) < 1e-12 and abs(rec.get("inner_tol", -1) - inner_tol) < 1e-15
            and rec.get("u_r", "f64") == u_r and rec.get("tiling") == tiling
            and rec.get("source_sha256") == kernel_sources_sha256())
    return rec if same else None


def hbm_calibration(dev):
    """Plain streaming rates on this GPU (torch kernels, 4 GiB buffers, far beyond the 256 MB
    Infinity Cache): a read-only reduction, a write-only fill, a copy and an add (two reads, one
    write: the read / write mix of the inner passes); best of 5 each, GB/s."""
    import torch
    nbytes = 1 << 32
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    c = torch.empty_like(a)
    a.fill_(1.0)
    b.fill_(0.0)
    torch.cuda.synchronize()

    def best(fn, moved):
        out = 0.0
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            out = max(out, moved / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        return out

    res = {"read_GBs": best(lambda: a.sum(), nbytes), "write_GBs": best(lambda: b.fill_(2.0), nbytes),
           "copy_GBs": best(lambda: b.copy_(a), 2 * nbytes),
           "add_GBs": best(lambda: torch.add(a, b, out=c), 3 * nbytes), "buffer_bytes": nbytes,
           "kernels": "torch sum (read), fill_ (write), copy_ (read + write), add (2 reads + write)"}
    del a, b, c
    torch.cuda.empty_cache()
    return res


def cpu_baseline(dim, ng, ng_sample, beta, alpha, mh, ms, sweeps, us, gpu_outer, normA, seconds=15.0):
    """Oracle (CPU, FP64 / emulated u_s) time per sweep on this workload's operator, extrapolated.

    The oracle runs `sweeps` sweeps (0: one sweep to size the sample, then as many as take about
    `seconds`) with the GPU's mean inner iteration counts on the grid of side ng_sample; below the
    full side its time per sweep is scaled by the unknown count (the oracle's work per sweep is
    linear in it)."""
    import workloads
    from threadpoolctl import threadpool_limits
    from oracle import gadi_ref, problems
    with threadpool_limits(1):
        spec = problems.convection_diffusion(dim, ng_sample, (beta,) * dim)
        A = problems.assemble(spec)
        xs = workloads.x_true(A.shape[0], 0, "normal" if dim == 3 else "uniform")
        b = A @ xs
        rh = gadi_ref.InnerRule(fixed=max(1, mh))
        rs = gadi_ref.InnerRule(fixed=max(1, ms))
        def run(k):
            t = time.perf_counter()
            gadi_ref.gadi(A, b, alpha, 1.0, normA=normA, max_outer=k, tol=0.0, prec=us, rule_h=rh, rule_s=rs,
                          stag_window=0, div_factor=0.0)
            return time.perf_counter() - t
        setup = run(0)                      # the oracle's set-up alone, subtracted below
        if sweeps <= 0:
            est = max(run(1) - setup, 1e-3)
            sweeps = int(max(1, min(500, round(seconds / est))))
        total = run(sweeps)
    per_sweep = max(total - setup, 1e-9) / sweeps
    scale = float(ng) ** dim / float(ng_sample) ** dim
    solve_s = per_sweep * scale * gpu_outer
    grid = "x".join([str(ng_sample)] * dim)
    what = (f"{sweeps} GADI sweep(s) ({per_sweep * sweeps:.1f} s) in the NumPy/SciPy oracle on the {grid} grid of this operator "
            f"(u_s={us} emulated, CG {mh} + CGNE {ms} iterations per sweep = the GPU's mean), "
            f"{per_sweep:.2f} s/sweep single-threaded")
    if scale != 1.0:
        what += f", scaled by the unknown count ({scale:.0f}x) to the full grid"
    what += f", extrapolated to the GPU's {gpu_outer} sweeps ({solve_s:.1f} s per solve)"
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": 1, "kind": "oracle", "sample": what,
            "scaled": scale != 1.0}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    from paper_2512_21164_amd import Problem, Solver, apply

    dim, ng, beta0, alpha0, itol0, desc, ng_cpu = WORKLOADS[args.workload]
    beta = beta0 if args.beta is None else args.beta
    inner_tol = itol0 if args.inner_tol is None else args.inner_tol
    pr = Problem.convection_diffusion(dim, ng, beta)
    alpha_source = "fixed"
    if args.alpha is None and alpha0 != "gpr":
        alpha = alpha0
    elif args.alpha is None or args.alpha == "gpr":
        from paper_2512_21164_amd.alpha_gpr import predict_alpha
        alpha = predict_alpha(pr, "f32" if args.us == "f64" else args.us)   # the model knows FP32 and BF16
        alpha_source = "gpr"
    else:
        alpha = float(args.alpha)
    n = pr.size
    dev = torch.device("cuda:0")
    calib = None if args.no_calib else hbm_calibration(dev)
    x_np = workloads.x_true(n, 0, "normal" if dim == 3 else "uniform")
    xt = torch.from_numpy(x_np).to(dev)
    del x_np
    b = apply(pr, xt)
    torch.cuda.synchronize()
    nxt = torch.linalg.norm(xt)

    def run(us, steps, warmup, alpha=alpha):
        fixed = {}
        if args.fixed_inner:
            fh, fs = (int(v) for v in args.fixed_inner.split(","))
            fixed = dict(fixed_inner_h=fh, fixed_inner_s=fs, stag_window=0, div_factor=0.0)
        s = Solver(pr, alpha=alpha, omega=1.0, u_s=us, u_r=args.u_r, tol=args.tol, max_outer=args.max_outer,
                   inner_tol_h=inner_tol, inner_tol_s=inner_tol, max_restarts=args.max_restarts,
                   tile_ry=args.tile_ry, tile_chunk=args.tile_chunk, autotune=args.autotune, normA=args.normA, **fixed)
        tiling = s.tiling
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
        return el, reps, fe, normA, tiling

    el, reps, fe, normA, tiling = run(args.us, args.steps, args.warmup)
    rep, hist = reps[-1]
    value = args.steps / el
    s_b = SBYTES[args.us]
    bytes_design = alg_bytes(hist, n, s_b, dim=dim, ry=tiling["ry"])
    bytes_unit = alg_bytes_unit(rep["outer"], rep["inner_h"], rep["inner_s"], n, s_b)
    kern_ms = float(np.mean([r["kernel_ms"] for r, _ in reps]))
    launches = float(np.mean([r["steps"] for r, _ in reps]))
    avg_launch_us = 1000.0 * kern_ms / launches
    achieved = (bytes_unit / launches) / (avg_launch_us * 1e-6) / 1e9
    achieved_design = (bytes_design / launches) / (avg_launch_us * 1e-6) / 1e9
    ry = tiling["ry"] if dim == 3 else 1

    out = {
        "metric": "time-to-1e-10 backward error & solves/s, mixed vs FP64 GADI; HBM GB/s",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"f64+{args.us}", "data": "synthetic",
        "config": {"workload": f"{desc}, beta=({','.join([str(beta)] * dim)}), "
                               f"alpha={alpha}, omega=1, inner tolerance {inner_tol}, target backward error {args.tol}"
                               + (", residual in FP64 pairs" if args.u_r == "f64x2" else ""),
                   "grid": [ng] * dim, "unknowns": n, "inner_precision": args.us, "alpha": alpha, "beta": beta,
                   "inner_tol": inner_tol, "residual_precision": args.u_r, "alpha_source": alpha_source,
                   "max_restarts": args.max_restarts, "tiling": tiling},
        "time_to_solution_s": el / args.steps,
        "mixed": {"u_s": args.us, "status": rep["status_name"], "outer": rep["outer"], "inner_h": rep["inner_h"],
                  "inner_s": rep["inner_s"], "be": rep["be"], "forward_error": fe, "solve_ms": rep["ms"],
                  "kernel_ms": rep["kernel_ms"], "launches": rep["steps"], "alg_bytes_per_solve": bytes_unit,
                  "alg_bytes_design_per_solve": bytes_design,
                  "alpha_final": rep["alpha"], "restarts": rep["restarts"]},
    }
    if args.fp64_steps > 0:
        el64, reps64, fe64, _, _ = run("f64", args.fp64_steps, args.fp64_warmup)
        r64, h64 = reps64[-1]
        out["fp64"] = {"solves_per_s": args.fp64_steps / el64, "time_to_solution_s": el64 / args.fp64_steps,
                       "status": r64["status_name"], "outer": r64["outer"], "inner_h": r64["inner_h"],
                       "inner_s": r64["inner_s"], "be": r64["be"], "forward_error": fe64,
                       "alg_bytes_per_solve": alg_bytes_unit(r64["outer"], r64["inner_h"], r64["inner_s"], n, 8),
                       "alg_bytes_design_per_solve": alg_bytes(h64, n, 8)}
        out["speedup_mixed_vs_fp64"] = value / out["fp64"]["solves_per_s"]
    if args.bf16_steps > 0 and args.us != "bf16":
        # the same workload with BF16-stored inner vectors (its own model alpha when alpha is the model's)
        a16 = alpha
        if alpha_source == "gpr":
            from paper_2512_21164_amd.alpha_gpr import predict_alpha
            a16 = predict_alpha(pr, "bf16")
        el16, reps16, fe16, _, _ = run("bf16", args.bf16_steps, args.bf16_warmup, alpha=a16)
        r16, _ = reps16[-1]
        out["bf16"] = {"solves_per_s": args.bf16_steps / el16, "time_to_solution_s": el16 / args.bf16_steps,
                       "alpha": a16, "status": r16["status_name"], "outer": r16["outer"], "inner_h": r16["inner_h"],
                       "inner_s": r16["inner_s"], "be": r16["be"], "forward_error": fe16}
        if "fp64" in out:
            out["speedup_bf16_vs_fp64"] = out["bf16"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    tname = {"bf16": "gadi::bf16", "f32": "float", "f64": "double"}[args.us]
    kname = f"gadi::gadi_step<{tname}, {dim}, {ry}, {'true' if args.u_r == 'f64x2' else 'false'}>"
    if any(r["restarts"] > 0 for r, _ in reps):
        # the sweep history holds the last attempt only: the bytes of a restarted solve are not known
        achieved = achieved_design = None
    rec = traffic_record(args.workload, args.us, alpha, beta, inner_tol, args.u_r, tiling)
    traffic = None
    if rec is not None and achieved_design is not None:
        traffic = float(rec["traffic_over_design"]) * bytes_design / launches
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
                       "traffic": traffic, "kernel": kname, "avg_launch_us": avg_launch_us,
                       "alg_bytes_per_launch": bytes_unit / launches,
                       "achieved_design": achieved_design,
                       "frac_design": achieved_design / HBM_PEAK_GBS if achieved_design is not None else None,
                       "design_bytes_per_launch": bytes_design / launches,
                       "traffic_over_design": float(rec["traffic_over_design"]) if rec is not None else None}
    if calib is not None:
        out["hbm_calibration"] = calib
    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu:
        print("[bench] CPU oracle baseline (bounded sample) ...", file=sys.stderr, flush=True)
        mh = int(round(rep["inner_h"] / max(1, rep["outer"])))
        ms = int(round(rep["inner_s"] / max(1, rep["outer"])))
        out["cpu_baseline"] = cpu_baseline(dim, ng, args.cpu_grid or ng_cpu, beta, alpha, mh, ms, args.cpu_sweeps,
                                           args.us, int(rep["outer"]), normA, args.cpu_seconds)
        if args.u_r != "f64":
            out["cpu_baseline"]["sample"] += "; the oracle forms the residual in FP64 (its exact residual is not timed)"
        print("[bench] CPU oracle baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
