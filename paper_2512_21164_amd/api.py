"""Python front end of the GADI library: problems, parameters, solver handles.

PyTorch provides device memory and streams only; every arithmetic step of a
solve runs in the HIP kernels of ``libgadi.so`` through the C ABI.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np

from . import _lib

PREC = _lib.PREC


@dataclasses.dataclass(frozen=True)
class Problem:
    """A 5/7-point constant-coefficient operator on an n[0] x n[1] (x n[2]) grid.

    (A u)_p = center u_p + sum_d (lo[d] u_{p-e_d} + hi[d] u_{p+e_d}) [+ i shift_im u_p],
    zero outside the grid, x-fastest ordering.
    """
    dim: int
    n: tuple
    center: float
    lo: tuple
    hi: tuple
    shift_im: float = 0.0
    is_complex: bool = False

    @property
    def size(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @staticmethod
    def convection_diffusion(dim: int, ng, beta, reaction: float = 0.0) -> "Problem":
        """-Lap u + beta . grad u + reaction u on the unit square/cube, centered
        differences with h = 1/(ng+1), scaled by h^2 (Sections 5.2, 5.3).

        ng may be an int or a per-axis tuple (then h differs per axis)."""
        ngs = tuple(int(v) for v in (ng if np.ndim(ng) else [ng] * dim))
        betas = tuple(float(v) for v in (beta if np.ndim(beta) else [beta] * dim))
        lo, hi = [], []
        for d in range(dim):
            h = 1.0 / (ngs[d] + 1)
            lo.append(-1.0 - 0.5 * betas[d] * h)
            hi.append(-1.0 + 0.5 * betas[d] * h)
        h0 = 1.0 / (ngs[0] + 1)
        while len(lo) < 3:
            lo.append(0.0)
            hi.append(0.0)
        n = ngs + (1,) * (3 - dim)
        return Problem(dim, n, 2.0 * dim + reaction * h0 * h0, tuple(lo), tuple(hi))

    @staticmethod
    def complex_reaction_diffusion(ng: int, sigma: float) -> "Problem":
        """-Lap u + i sigma u on the unit square, times h^2 (Section 5.4, constant potential)."""
        h = 1.0 / (ng + 1)
        return Problem(2, (ng, ng, 1), 4.0, (-1.0, -1.0, 0.0), (-1.0, -1.0, 0.0),
                       shift_im=sigma * h * h, is_complex=True)

    def c_struct(self) -> _lib.gadi_stencil:
        s = _lib.gadi_stencil()
        s.dim = self.dim
        s.is_complex = 1 if self.is_complex else 0
        for i in range(3):
            s.n[i] = int(self.n[i])
            s.lo[i] = float(self.lo[i])
            s.hi[i] = float(self.hi[i])
        s.center = float(self.center)
        s.shift_im = float(self.shift_im)
        return s


def make_params(**kw) -> _lib.gadi_params:
    """gadi_params from keyword arguments over the library defaults.

    u_s and u_r may be given as "f64", "f32", "bf16", "f64x2" or a GADI_*
    constant.
    """
    lib = _lib.load()
    p = _lib.gadi_params()
    lib.gadi_params_default(C.byref(p))
    for k, v in kw.items():
        if k in ("u_s", "u_r", "u") and isinstance(v, str):
            v = PREC[v]
        if not hasattr(p, k):
            raise KeyError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dtype(problem: Problem):
    import torch
    return torch.complex128 if problem.is_complex else torch.float64


def workspace_bytes(problem: Problem, params: _lib.gadi_params) -> int:
    lib = _lib.load()
    out = C.c_size_t(0)
    _lib.check(lib.gadi_workspace_bytes(C.byref(problem.c_struct()), C.byref(params), C.byref(out)),
               "gadi_workspace_bytes")
    return int(out.value)


class Solver:
    """A gadi_handle with its workspace (a torch uint8 tensor on the device)."""

    def __init__(self, problem: Problem, stream=None, device="cuda", workspace=None, autotune: bool = False,
                 **params):
        """autotune: before sizing the workspace, let the library time the tile shapes of this
        problem's class (once per class and process, see ``autotune``) unless tile_ry or a
        positive tile_chunk is given (tile_chunk = -k takes the tuned chunk k times longer)."""
        import torch
        self.lib = _lib.load()
        if autotune and not params.get("tile_ry") and (params.get("tile_chunk") or 0) <= 0:
            autotune_class(problem, stream=stream, device=device, **params)
        self.problem = problem
        self.params = make_params(**params)
        self.stream = stream
        self._st = problem.c_struct()
        nbytes = workspace_bytes(problem, self.params)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        elif workspace.numel() < nbytes:
            raise ValueError("workspace too small")
        self.workspace = workspace
        self.handle = C.c_void_p()
        _lib.check(self.lib.gadi_create(C.byref(self._st), C.byref(self.params),
                                        C.c_void_p(_stream_handle(stream)),
                                        C.c_void_p(workspace.data_ptr()),
                                        C.c_size_t(workspace.numel()), C.byref(self.handle)),
                   "gadi_create")

    @property
    def normA(self) -> float:
        v = C.c_double(0)
        _lib.check(self.lib.gadi_get_norm(self.handle, C.byref(v)), "gadi_get_norm")
        return v.value

    @property
    def tiling(self) -> dict:
        """Tile shape of the handle's step kernel: rows per wave (ry), planes per chunk of the
        inner and FP64 tilings, and blocks of the larger tiling."""
        v = (C.c_int32 * 4)()
        _lib.check(self.lib.gadi_get_tiling(self.handle, v), "gadi_get_tiling")
        return {"ry": v[0], "chunk_inner": v[1], "chunk_fp64": v[2], "tiles": v[3]}

    def set_params(self, **params):
        p = make_params(**params)
        _lib.check(self.lib.gadi_set_params(self.handle, C.byref(p)), "gadi_set_params")
        self.params = p

    def _hist_buf(self, history: bool):
        if not history:
            return None, None
        n = 4 * (int(self.params.max_outer) + 1)
        buf = np.zeros(n, dtype=np.float64)
        return buf, buf.ctypes.data_as(C.POINTER(C.c_double))

    def solve(self, b, x=None, history: bool = False):
        """Solve A x = b; returns (x, report dict[, history array (k, 4)]).

        The history covers the last attempt when alpha restarts happened."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        self._check_vec(b)
        self._check_vec(x)
        rep = _lib.gadi_report()
        buf, ptr = self._hist_buf(history)
        st = _lib.check(self.lib.gadi_solve(self.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                            C.byref(rep), ptr), "gadi_solve")
        out = rep.as_dict()
        out["status_name"] = self.lib.gadi_status_string(st).decode()
        if history:
            k = int(rep.attempt_outer) + 1
            return x, out, buf[: 4 * k].reshape(k, 4)
        return x, out

    def solve_async(self, b, x):
        self._check_vec(b)
        self._check_vec(x)
        _lib.check(self.lib.gadi_solve_async(self.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr())),
                   "gadi_solve_async")

    def query(self, wait: bool = False):
        rep = _lib.gadi_report()
        st = _lib.check(self.lib.gadi_query(self.handle, 1 if wait else 0, C.byref(rep), None), "gadi_query")
        if st == _lib.GADI_RUNNING:
            return None
        out = rep.as_dict()
        out["status_name"] = self.lib.gadi_status_string(st).decode()
        return out

    def _check_vec(self, v):
        if not v.is_cuda or v.dtype != _dtype(self.problem) or not v.is_contiguous() or v.numel() != self.problem.size:
            raise ValueError(f"expected a contiguous {_dtype(self.problem)} CUDA tensor of {self.problem.size} values")

    def close(self):
        if self.handle:
            self.lib.gadi_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_dense(problem: Problem, *vs):
    """Every vector a dense utility kernel touches must hold the whole grid."""
    for v in vs:
        if not v.is_cuda or v.dtype != _dtype(problem) or not v.is_contiguous() or v.numel() != problem.size:
            raise ValueError(f"expected a contiguous {_dtype(problem)} CUDA tensor of {problem.size} values")


def apply(problem: Problem, x, transpose: bool = False, stream=None):
    """y = A x (or A^H x) on the device."""
    import torch
    lib = _lib.load()
    _check_dense(problem, x)
    y = torch.empty_like(x)
    _lib.check(lib.gadi_apply(C.byref(problem.c_struct()), C.c_void_p(_stream_handle(stream)),
                              C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 1 if transpose else 0),
               "gadi_apply")
    return y


def residual(problem: Problem, b, x, u_r="f64", stream=None):
    """r = b - A x on the device, in FP64 (u_r = "f64") or extra precision ("f64x2")."""
    import torch
    lib = _lib.load()
    _check_dense(problem, b, x)
    r = torch.empty_like(x)
    _lib.check(lib.gadi_residual(C.byref(problem.c_struct()), C.c_void_p(_stream_handle(stream)),
                                 C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(r.data_ptr()),
                                 PREC[u_r] if isinstance(u_r, str) else int(u_r)),
               "gadi_residual")
    return r


def solve_noalloc(problem: Problem, b, x=None, history: bool = False, stream=None, **params):
    """One solve through gadi_solve_noalloc: the library's static device workspace, no allocation
    by the library (x is allocated here only when not given).  Returns (x, report[, history])."""
    import torch
    lib = _lib.load()
    if x is None:
        x = torch.zeros_like(b)
    _check_dense(problem, b, x)
    p = make_params(**params)
    rep = _lib.gadi_report()
    buf = ptr = None
    if history:
        buf = np.zeros(4 * (int(p.max_outer) + 1), dtype=np.float64)
        ptr = buf.ctypes.data_as(C.POINTER(C.c_double))
    st = _lib.check(lib.gadi_solve_noalloc(C.byref(problem.c_struct()), C.byref(p),
                                           C.c_void_p(_stream_handle(stream)), C.c_void_p(b.data_ptr()),
                                           C.c_void_p(x.data_ptr()), C.byref(rep), ptr), "gadi_solve_noalloc")
    out = rep.as_dict()
    out["status_name"] = lib.gadi_status_string(st).decode()
    if history:
        k = int(rep.attempt_outer) + 1
        return x, out, buf[: 4 * k].reshape(k, 4)
    return x, out


def autotune(problem: Problem, b, x, stream=None, **params):
    """Choose (tile_ry, tile_chunk) for this problem's class by timing whole sweeps on the device
    (gadi_autotune); returns (ry, chunk, microseconds per sweep, or -1 when the class was tuned
    already).  Handles created afterwards without an explicit tile shape use the choice."""
    import torch
    lib = _lib.load()
    p = make_params(**params)
    worst = make_params(**dict(params, tile_chunk=2, tile_ry=1))
    nbytes = workspace_bytes(problem, worst)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    ry, ch, us = C.c_int32(0), C.c_int32(0), C.c_double(0)
    _lib.check(lib.gadi_autotune(C.byref(problem.c_struct()), C.byref(p), C.c_void_p(_stream_handle(stream)),
                                 C.c_void_p(ws.data_ptr()), C.c_size_t(nbytes), C.c_void_p(b.data_ptr()),
                                 C.c_void_p(x.data_ptr()), C.byref(ry), C.byref(ch), C.byref(us)),
               "gadi_autotune")
    torch.cuda.current_stream(b.device).synchronize() if stream is None else stream.synchronize()
    del ws
    return ry.value, ch.value, us.value


def autotune_class(problem: Problem, stream=None, device="cuda", **params):
    """Tune the tile shape of this problem's class on a synthetic right-hand side b = A 1
    (nothing is read from or written to caller data); see ``autotune``."""
    import torch
    ones = torch.ones(problem.size, dtype=_dtype(problem), device=device)
    b = apply(problem, ones, stream=stream)
    x = torch.zeros_like(b)
    return autotune(problem, b, x, stream=stream, **params)


__all__ = ["Problem", "Solver", "make_params", "apply", "autotune", "autotune_class", "solve_noalloc",
           "workspace_bytes"]
