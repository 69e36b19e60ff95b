"""Data-driven initial alpha (Section 4.2): training data, fit and prediction.

Section 4.3's selection procedure starts from an alpha predicted by a
Gaussian-process regression (GPR) model trained once on small, cheap
problems of an equation family and reused for large ones.  This module

* ``collect``: runs the library's solver on the small training problems over
  a log-spaced alpha grid (GPU) and records the iteration counts;
* ``best_log_alpha``: the best alpha of one problem, by the algorithmic bytes
  the solve moves (outer sweeps and inner iterations weighted by their bytes
  per unknown, the quantity that sets the time of large, bandwidth-bound
  solves; small training solves are launch-bound, so their wall time would
  mislead), refined by a parabola through the grid minimum in log-log;
* ``fit``: the GPR hyperparameters by maximising the log marginal likelihood;
* ``Model`` / ``predict_alpha``: prediction through the C ABI
  (gadi_alpha_features, gadi_alpha_gpr_*).

The packaged model ``alpha_gpr_model.json`` was trained with ``collect`` and
``fit`` on the problems of ``TRAIN_SET`` (FP32 and BF16 inner solves, inner
tolerance 1e-2, target backward error 1e-10).

    python -m paper_2512_21164_amd.alpha_gpr collect OUT.json      (GPU)
    python -m paper_2512_21164_amd.alpha_gpr fit IN.json MODEL.json
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

from . import _lib
from .api import PREC, Problem

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "alpha_gpr_model.json")

# log-spaced alpha grid, four values per decade
ALPHAS = [float(10.0 ** (e / 4.0)) for e in range(-16, 5)]
TRAIN_PRECS = ("f32", "bf16")
INNER_TOL = 1e-2
TOL = 1e-10
MAX_OUTER = 4000


def train_set():
    """(name, Problem) pairs of the training families: 2D and 3D convection-diffusion
    (Sections 5.2, 5.3) and the complex reaction-diffusion problem (Section 5.4)."""
    out = []
    for ng in (48, 96, 192, 384, 768, 1536):
        for beta in (1.0, 10.0, 100.0):
            out.append((f"cd2_{ng}_b{beta:g}", Problem.convection_diffusion(2, ng, beta)))
    for ng in (12, 24, 48, 96):
        for beta in (1.0, 10.0, 100.0):
            out.append((f"cd3_{ng}_b{beta:g}", Problem.convection_diffusion(3, ng, beta)))
    for ng in (48, 96, 192, 384, 768, 1536):
        for sigma in (10.0, 100.0, 1000.0):
            out.append((f"crd_{ng}_s{sigma:g}", Problem.complex_reaction_diffusion(ng, sigma)))
    return out


def features(problem: Problem, u_s) -> np.ndarray:
    lib = _lib.load()
    f = (C.c_double * 4)()
    st = problem.c_struct()
    _lib.check(lib.gadi_alpha_features(C.byref(st), PREC[u_s] if isinstance(u_s, str) else int(u_s), f),
               "gadi_alpha_features")
    return np.array(list(f))


def solve_cost(rep: dict, u_s: str, cplx: bool) -> float:
    """Algorithmic bytes per unknown of a finished solve: an outer sweep moves 3 FP64 and
    3 u_s words per unknown, a CG or CGNE iteration 8 u_s words (complex doubles both)."""
    w = 16 if cplx else 8
    s = {"f64": 8, "f32": 4, "bf16": 2}[u_s] * (2 if cplx else 1)
    return rep["outer"] * (3 * w + 3 * s) + (rep["inner_h"] + rep["inner_s"]) * 8 * s


def best_log_alpha(alphas, costs):
    """log10 of the best alpha: grid minimum of the cost, refined by the vertex of the parabola
    through the minimum and its two neighbours (log10 alpha against log10 cost), kept within
    half a grid step.  None if no alpha converged."""
    la = np.log10(np.asarray(alphas, dtype=np.float64))
    c = np.asarray(costs, dtype=np.float64)
    ok = np.isfinite(c)
    if not ok.any():
        return None
    i = int(np.argmin(np.where(ok, c, np.inf)))
    if 0 < i < len(c) - 1 and ok[i - 1] and ok[i + 1]:
        y0, y1, y2 = np.log10(c[i - 1]), np.log10(c[i]), np.log10(c[i + 1])
        den = y0 - 2.0 * y1 + y2
        if den > 0:
            step = la[i + 1] - la[i]
            shift = 0.5 * step * (y0 - y2) / den
            return float(la[i] + np.clip(shift, -0.5 * step, 0.5 * step))
    return float(la[i])


def _scan(run, alphas, start: int, patience: int = 2):
    """Costs over the grid, walked from index ``start`` upwards and then downwards; each walk
    stops after ``patience`` consecutive values worse than the best so far (the cost is
    unimodal in log alpha: the contraction improves and then the inner solves or the
    sweep count take over).  Unvisited grid points stay None."""
    costs = [None] * len(alphas)
    best = math.inf
    for direction in (+1, -1):
        worse = 0
        i = start if direction > 0 else start - 1
        while 0 <= i < len(alphas) and worse < patience:
            c = run(alphas[i], best)
            costs[i] = c
            if c < best:
                best, worse = c, 0
            else:
                worse += 1
            i += direction
    return costs


def collect(out_path: str, problems=None, precs=TRAIN_PRECS, alphas=ALPHAS, seed: int = 0):
    """Solve every training problem over the alpha grid (GPU) and write the records.

    The walk starts at the grid value nearest sqrt(lambda_min(M) lambda_max(M)), the alpha
    that minimises the contraction bound of exact GADI, and a solve may take at most eight
    times the sweeps of the best solve so far (the cost of a solve that needs more is
    recorded as infinite)."""
    import torch

    import workloads
    from .api import Solver, apply
    problems = problems or train_set()
    records = []
    t0 = time.time()
    la_grid = np.log10(np.asarray(alphas))
    for name, pr in problems:
        n = pr.size
        if pr.is_complex:
            b = torch.from_numpy(workloads.complex_rhs(n, seed)).to("cuda")
        else:
            xt = torch.from_numpy(workloads.x_true(n, seed)).to("cuda")
            b = apply(pr, xt)
        for us in precs:
            f = features(pr, us)
            start = int(np.argmin(np.abs(la_grid - 0.5 * (f[0] + f[1]))))
            kw = dict(u_s=us, tol=TOL, inner_tol_h=INNER_TOL, inner_tol_s=INNER_TOL)
            s = Solver(pr, alpha=alphas[start], max_outer=MAX_OUTER, **kw)
            runs = {}
            best_outer = [MAX_OUTER]

            def run(a, best_cost):
                cap = min(MAX_OUTER, 8 * best_outer[0]) if math.isfinite(best_cost) else MAX_OUTER
                s.set_params(alpha=a, max_outer=cap, **kw)
                x = torch.zeros_like(b)
                _, rep = s.solve(b, x)
                ok = rep["status"] == _lib.GADI_OK
                c = solve_cost(rep, us, pr.is_complex) if ok else math.inf
                runs[a] = [int(rep["outer"]), int(rep["inner_h"]), int(rep["inner_s"]), int(rep["status"])]
                if ok and c < best_cost:
                    best_outer[0] = int(rep["outer"])
                return c

            costs = _scan(run, alphas, start)
            s.close()
            la = best_log_alpha(alphas, [math.inf if c is None else c for c in costs])
            rec = {"name": name, "u_s": us, "features": f.tolist(), "alphas": alphas,
                   "costs": [c if (c is not None and math.isfinite(c)) else None for c in costs],
                   "visited": [c is not None for c in costs],
                   "runs": {repr(a): v for a, v in runs.items()}, "best_log10_alpha": la}
            records.append(rec)
            print(f"[alpha_gpr] {name} {us}: {len(runs)} solves, best alpha "
                  f"{10 ** la if la is not None else None} ({time.time() - t0:.0f} s)", flush=True)
    with open(out_path, "w") as fh:
        json.dump({"inner_tol": INNER_TOL, "tol": TOL, "max_outer": MAX_OUTER, "records": records}, fh)
    return records


def _log_marginal(theta, X, y):
    """Log marginal likelihood of the GPR with a linear mean under a flat prior
    (Rasmussen and Williams 2006, eq. 2.45), theta = log(l_0..l_3, sf, sn)."""
    ell = np.exp(theta[:4])
    sf, sn = np.exp(theta[4]), np.exp(theta[5])
    d2 = (((X[:, None, :] - X[None, :, :]) / ell) ** 2).sum(axis=2)
    Ky = sf * sf * np.exp(-0.5 * d2) + (sn * sn + 1e-10) * np.eye(len(X))
    try:
        L = np.linalg.cholesky(Ky)
    except np.linalg.LinAlgError:
        return -np.inf
    H = np.column_stack([np.ones(len(X)), X])
    Li_y = np.linalg.solve(L, y)
    Li_H = np.linalg.solve(L, H)
    A = Li_H.T @ Li_H
    try:
        LA = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return -np.inf
    z = np.linalg.solve(LA, Li_H.T @ Li_y)
    n, m = len(X), H.shape[1]
    return float(-0.5 * Li_y @ Li_y + 0.5 * z @ z - np.sum(np.log(np.diag(L))) - np.sum(np.log(np.diag(LA)))
                 - 0.5 * (n - m) * np.log(2 * np.pi))


def usable(rec) -> bool:
    """A record's optimum is a target only if it converged and its best grid value is interior
    (an optimum at the end of the grid is censored: the true best alpha lies beyond it)."""
    if rec["best_log10_alpha"] is None:
        return False
    c = [math.inf if v is None else v for v in rec["costs"]]
    i = int(np.argmin(c))
    return 0 < i < len(c) - 1


def fit(records, restarts: int = 8, seed: int = 0):
    """Hyperparameters (l_0..l_3, sf, sn) maximising the log marginal likelihood (L-BFGS-B
    over their logarithms from several starts).  Returns (X, y, hyper)."""
    from scipy.optimize import minimize
    rows = [r for r in records if usable(r)]
    X = np.array([r["features"] for r in rows], dtype=np.float64)
    y = np.array([r["best_log10_alpha"] for r in rows], dtype=np.float64)
    span = np.maximum(X.max(axis=0) - X.min(axis=0), 1e-3)
    rng = np.random.default_rng(seed)
    best = None
    for k in range(restarts):
        th0 = np.concatenate([np.log(span * rng.uniform(0.3, 3.0, 4)), [np.log(rng.uniform(0.05, 0.5)),
                                                                     np.log(rng.uniform(0.02, 0.2))]])
        res = minimize(lambda t: -_log_marginal(t, X, y), th0, method="L-BFGS-B",
                       bounds=[(np.log(s * 0.05), np.log(s * 100.0)) for s in span] + [(np.log(1e-3), np.log(10.0)),
                                                                                        (np.log(1e-3), np.log(1.0))])
        if np.isfinite(res.fun) and (best is None or res.fun < best.fun):
            best = res
    hyper = np.exp(best.x)
    return X, y, hyper


class Model:
    """A trained GPR model held by the C library."""

    def __init__(self, X, y, hyper):
        self.lib = _lib.load()
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        self.hyper = np.ascontiguousarray(hyper, dtype=np.float64)
        if self.X.ndim != 2 or self.X.shape[1] != 4 or len(self.y) != len(self.X) or len(self.hyper) != 6:
            raise ValueError("X must be n x 4, y of length n, hyper of length 6")
        D = C.POINTER(C.c_double)
        self.handle = C.c_void_p()
        _lib.check(self.lib.gadi_alpha_gpr_create(len(self.y), self.X.ctypes.data_as(D), self.y.ctypes.data_as(D),
                                                  self.hyper.ctypes.data_as(D), C.byref(self.handle)),
                   "gadi_alpha_gpr_create")

    @staticmethod
    def load(path: str = MODEL_PATH) -> "Model":
        with open(path) as fh:
            m = json.load(fh)
        return Model(m["X"], m["y"], m["hyper"])

    def predict_features(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        D = C.POINTER(C.c_double)
        mu, sd = C.c_double(0), C.c_double(0)
        _lib.check(self.lib.gadi_alpha_gpr_predict(self.handle, f.ctypes.data_as(D), C.byref(mu), C.byref(sd)),
                   "gadi_alpha_gpr_predict")
        return mu.value, sd.value

    def predict(self, problem: Problem, u_s):
        """(alpha, sd of log10 alpha) for a problem and inner precision."""
        mu, sd = self.predict_features(features(problem, u_s))
        return 10.0 ** mu, sd

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.gadi_alpha_gpr_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def predict_alpha(problem: Problem, u_s="f32"):
    """alpha from the packaged model (Section 4.3, step 1)."""
    return Model.load().predict(problem, u_s)[0]


def main(argv):
    if len(argv) >= 2 and argv[0] == "collect":
        collect(argv[1])
    elif len(argv) >= 3 and argv[0] == "fit":
        with open(argv[1]) as fh:
            data = json.load(fh)
        X, y, hyper = fit(data["records"])
        with open(argv[2], "w") as fh:
            json.dump({"features": ["log10 lambda_min(M)", "log10 lambda_max(M)", "log10 max(rho(N),1e-12)",
                                    "log10 u_s"], "target": "log10 alpha_opt",
                       "hyper": hyper.tolist(), "X": X.tolist(), "y": y.tolist(),
                       "trained_on": [f"{r['name']}:{r['u_s']}" for r in data["records"] if usable(r)],
                       "inner_tol": data["inner_tol"], "tol": data["tol"]}, fh, indent=1)
        print(f"fit: hyper = {hyper}")
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
