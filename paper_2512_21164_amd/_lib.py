"""ctypes binding of the C ABI in include/gadi.h (argument marshalling only).

Every function keeps the C name and signature; device buffers are passed as
integer addresses (for example ``tensor.data_ptr()``) and streams as the
integer ``torch.cuda.current_stream().cuda_stream``.  The library is the
in-tree ``libgadi.so`` built by ``paper_2512_21164_amd.build``; loading fails
loudly when it is missing, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgadi.so")

GADI_OK, GADI_NOT_CONVERGED, GADI_STAGNATED, GADI_DIVERGED, GADI_RUNNING = 0, 1, 2, 3, 4
GADI_ERR_INVALID_ARG, GADI_ERR_UNSUPPORTED, GADI_ERR_WORKSPACE = -1, -2, -3
GADI_ERR_HIP, GADI_ERR_CAPACITY, GADI_ERR_STATE = -4, -5, -6
GADI_F64, GADI_F32, GADI_BF16, GADI_F64X2 = 0, 1, 2, 3
PREC = {"f64": GADI_F64, "f32": GADI_F32, "bf16": GADI_BF16, "f64x2": GADI_F64X2}


class gadi_stencil(C.Structure):
    _fields_ = [("dim", C.c_int32), ("is_complex", C.c_int32), ("n", C.c_int64 * 3),
                ("center", C.c_double), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("shift_im", C.c_double)]


class gadi_params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("omega", C.c_double),
                ("u_r", C.c_int32), ("u", C.c_int32), ("u_s", C.c_int32),
                ("stop_on_relres", C.c_int32), ("tol", C.c_double), ("max_outer", C.c_int64),
                ("stag_window", C.c_int32), ("inner_stag_window", C.c_int32),
                ("div_factor", C.c_double), ("inner_tol_h", C.c_double), ("inner_tol_s", C.c_double),
                ("max_inner_h", C.c_int32), ("max_inner_s", C.c_int32),
                ("fixed_inner_h", C.c_int32), ("fixed_inner_s", C.c_int32),
                ("normA", C.c_double), ("norm_iters", C.c_int32),
                ("tile_ry", C.c_int32), ("tile_chunk", C.c_int32), ("max_restarts", C.c_int32),
                ("safeguard_tau", C.c_double), ("alpha_growth", C.c_double)]


class gadi_report(C.Structure):
    _fields_ = [("outer", C.c_int64), ("inner_h", C.c_int64), ("inner_s", C.c_int64),
                ("be", C.c_double), ("relres", C.c_double), ("normA", C.c_double),
                ("normb", C.c_double), ("ms", C.c_double), ("kernel_ms", C.c_double),
                ("status", C.c_int32), ("steps", C.c_int32),
                ("alpha", C.c_double), ("restarts", C.c_int32), ("attempt_outer", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_S = C.POINTER(gadi_stencil)
_PP = C.POINTER(gadi_params)
_R = C.POINTER(gadi_report)
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)

# (name, restype, argtypes) of every exported C function
SIGNATURES = [
    ("gadi_version", C.c_char_p, []),
    ("gadi_status_string", C.c_char_p, [C.c_int32]),
    ("gadi_last_error", C.c_char_p, []),
    ("gadi_params_default", None, [_PP]),
    ("gadi_workspace_bytes", C.c_int32, [_S, _PP, C.POINTER(C.c_size_t)]),
    ("gadi_create", C.c_int32, [_S, _PP, _P, _P, C.c_size_t, C.POINTER(_P)]),
    ("gadi_set_params", C.c_int32, [_P, _PP]),
    ("gadi_condition_estimate", C.c_int32, [_S, C.c_double, _D, _D]),
    ("gadi_solve", C.c_int32, [_P, _P, _P, _R, _D]),
    ("gadi_solve_async", C.c_int32, [_P, _P, _P]),
    ("gadi_query", C.c_int32, [_P, C.c_int32, _R, _D]),
    ("gadi_get_norm", C.c_int32, [_P, _D]),
    ("gadi_get_tiling", C.c_int32, [_P, _I]),
    ("gadi_destroy", C.c_int32, [_P]),
    ("gadi_apply", C.c_int32, [_S, _P, _P, _P, C.c_int32]),
    ("gadi_residual", C.c_int32, [_S, _P, _P, _P, _P, C.c_int32]),
    ("gadi_alpha_features", C.c_int32, [_S, C.c_int32, _D]),
    ("gadi_alpha_gpr_create", C.c_int32, [C.c_int32, _D, _D, _D, C.POINTER(_P)]),
    ("gadi_alpha_gpr_predict", C.c_int32, [_P, _D, _D, _D]),
    ("gadi_alpha_gpr_destroy", C.c_int32, [_P]),
    ("gadi_batch_workspace_bytes", C.c_int32, [C.c_int32, C.POINTER(C.c_size_t)]),
    ("gadi_batch_create", C.c_int32, [C.c_int32, _P, _P, C.c_size_t, C.POINTER(_P)]),
    ("gadi_batch_add", C.c_int32, [_P, _P, _P, _P, _I]),
    ("gadi_batch_step", C.c_int32, [_P, C.c_int32]),
    ("gadi_batch_poll", C.c_int32, [_P, _I, _I]),
    ("gadi_batch_remove", C.c_int32, [_P, C.c_int32, _R, _D]),
    ("gadi_batch_destroy", C.c_int32, [_P]),
    ("gadi_autotune", C.c_int32, [_S, _PP, _P, _P, C.c_size_t, _P, _P, _I, _I, _D]),
    ("gadi_solve_noalloc", C.c_int32, [_S, _PP, _P, _P, _P, _R, _D]),
]
# device bytes of the allocation-free solve's static workspace (GADI_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None


def load(path: str = LIB_PATH):
    """Load libgadi.so and declare the signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run paper_2512_21164_amd.build.build())")
    # torch first: its HIP runtime is then the one the library binds to, so tensors and
    # streams from torch and the library's launches share one runtime in the process
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GadiError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.gadi_last_error().decode()
        super().__init__(f"{where}: {lib.gadi_status_string(status).decode()} ({status}) {msg}")
        self.status = status


def check(status: int, where: str) -> int:
    """Raise GadiError for negative (error) statuses, return the status otherwise."""
    if status < 0:
        raise GadiError(status, where)
    return status
