"""The C-ABI library loads and exports every declared symbol; host-side checks.

No device work is issued here: only calls that validate arguments before
touching the GPU (workspace sizing, argument errors, defaults, strings).
"""
import ctypes as C
import os
import re

import pytest

from paper_2512_21164_amd import _lib, api

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gadi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gadi_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(names) == bound


def test_defaults_and_strings():
    lib = _lib.load()
    p = api.make_params()
    assert p.alpha == 0.5 and p.omega == 1.0 and p.tol == 1e-10 and p.u_s == _lib.GADI_F64
    assert p.max_outer == 20000 and p.stag_window == 200 and p.inner_stag_window == 20
    assert p.max_restarts == 0 and p.safeguard_tau == 0.0 and p.alpha_growth == pytest.approx(10 ** (3 / 7), rel=1e-15)
    assert lib.gadi_status_string(0) == b"OK"
    assert lib.gadi_status_string(-3) == b"ERR_WORKSPACE"
    assert lib.gadi_version().startswith(b"gadi")


def _ws(problem, **kw):
    return api.workspace_bytes(problem, api.make_params(**kw))


def test_workspace_size_scales_with_precision():
    pr = api.Problem.convection_diffusion(2, 256, 10.0)
    n = 256 * 256
    w64, w32, w16 = (_ws(pr, u_s=u) for u in ("f64", "f32", "bf16"))
    assert w64 > w32 > w16
    assert w64 - w32 >= 4 * 4 * n * 0.99 and w32 - w16 >= 4 * 2 * n * 0.99
    assert w16 >= 3 * 8 * n


@pytest.mark.parametrize("bad", [dict(alpha=0.0), dict(alpha=-1.0), dict(omega=2.0), dict(omega=-0.1),
                                 dict(u_r=1), dict(u_r=4), dict(u=2), dict(u=3), dict(u_s=3), dict(u_s=7),
                                 dict(max_inner_h=0),
                                 dict(tile_ry=3), dict(tol=-1.0), dict(normA=-1.0), dict(max_restarts=-1),
                                 dict(alpha_growth=1.0), dict(u_s="bf16", safeguard_tau=1e-3),
                                 dict(safeguard_tau=-1.0), dict(tile_chunk=-65), dict(tile_chunk=4097)])
def test_argument_errors(bad):
    pr = api.Problem.convection_diffusion(2, 32, 1.0)
    with pytest.raises(_lib.GadiError):
        _ws(pr, **bad)


def test_tile_share_means_fewer_tiles():
    """tile_chunk = -k: chunks k times longer, so fewer tiles and fewer reduction partials in the
    workspace (the vectors are the same size)."""
    pr = api.Problem.convection_diffusion(2, 1024, 3.0)
    base = _ws(pr, u_s="f32")
    shares = [_ws(pr, u_s="f32", tile_chunk=-k) for k in (2, 8, 64)]
    assert base >= shares[0] >= shares[1] >= shares[2]
    assert base > shares[2]


def test_extra_precision_residual_is_accepted_and_sized_like_fp64():
    pr = api.Problem.convection_diffusion(2, 96, 3.0)
    for us in ("f64", "f32", "bf16"):
        assert _ws(pr, u_s=us, u_r="f64x2") == _ws(pr, u_s=us, u_r="f64")


def test_residual_argument_errors():
    """gadi_residual validates before any device work (the pointers are never used)."""
    lib = _lib.load()
    st = api.Problem.convection_diffusion(2, 16, 1.0).c_struct()
    p1, p2, p3 = C.c_void_p(16), C.c_void_p(32), C.c_void_p(48)
    assert lib.gadi_residual(C.byref(st), None, p1, p2, p3, 7) == _lib.GADI_ERR_INVALID_ARG
    assert lib.gadi_residual(C.byref(st), None, p1, p2, p3, _lib.GADI_F32) == _lib.GADI_ERR_INVALID_ARG
    assert lib.gadi_residual(C.byref(st), None, p1, p2, p1, _lib.GADI_F64X2) == _lib.GADI_ERR_INVALID_ARG
    assert lib.gadi_residual(C.byref(st), None, p1, p2, p2, _lib.GADI_F64) == _lib.GADI_ERR_INVALID_ARG
    assert lib.gadi_residual(C.byref(st), None, None, p2, p3, _lib.GADI_F64X2) == _lib.GADI_ERR_INVALID_ARG
    assert lib.gadi_residual(None, None, p1, p2, p3, _lib.GADI_F64X2) == _lib.GADI_ERR_INVALID_ARG
    flat = api.Problem(2, (8, 8, 2), 4.0, (-1, -1, 0), (-1, -1, 0)).c_struct()
    assert lib.gadi_residual(C.byref(flat), None, p1, p2, p3, _lib.GADI_F64X2) == _lib.GADI_ERR_INVALID_ARG


def test_problem_errors():
    lib = _lib.load()
    p = api.make_params()
    out = C.c_size_t(0)
    bad_dim = api.Problem(4, (4, 4, 4), 4.0, (-1, -1, -1), (-1, -1, -1))
    assert lib.gadi_workspace_bytes(C.byref(bad_dim.c_struct()), C.byref(p), C.byref(out)) == _lib.GADI_ERR_INVALID_ARG
    cplx_conv = api.Problem(2, (8, 8, 1), 4.0, (-1.1, -1.0, 0), (-0.9, -1.0, 0), shift_im=0.1, is_complex=True)
    assert lib.gadi_workspace_bytes(C.byref(cplx_conv.c_struct()), C.byref(p), C.byref(out)) == _lib.GADI_ERR_UNSUPPORTED
    flat = api.Problem(2, (8, 8, 2), 4.0, (-1, -1, 0), (-1, -1, 0))
    assert lib.gadi_workspace_bytes(C.byref(flat.c_struct()), C.byref(p), C.byref(out)) == _lib.GADI_ERR_INVALID_ARG


def test_create_rejects_before_device_work():
    lib = _lib.load()
    pr = api.Problem.convection_diffusion(2, 32, 1.0)
    p = api.make_params()
    h = C.c_void_p()
    st = pr.c_struct()
    assert lib.gadi_create(C.byref(st), C.byref(p), None, None, 0, C.byref(h)) == _lib.GADI_ERR_WORKSPACE
    assert lib.gadi_create(C.byref(st), C.byref(p), None, C.c_void_p(256), 16, C.byref(h)) == _lib.GADI_ERR_WORKSPACE
    assert lib.gadi_create(C.byref(st), C.byref(p), None, C.c_void_p(300), 1 << 40, C.byref(h)) == _lib.GADI_ERR_WORKSPACE
    assert b"aligned" in lib.gadi_last_error()
    assert not h.value
    assert lib.gadi_batch_create(0, None, None, 0, C.byref(h)) == _lib.GADI_ERR_INVALID_ARG


def test_problem_discretization_matches_pde_coefficients():
    pr = api.Problem.convection_diffusion(3, 9, (10.0, 0.0, -10.0))
    h = 0.1
    assert pr.center == 6.0
    assert pr.lo == (-1 - 0.5 * 10 * h, -1.0, -1 + 0.5 * 10 * h)
    assert pr.hi == (-1 + 0.5 * 10 * h, -1.0, -1 - 0.5 * 10 * h)
    c = api.Problem.complex_reaction_diffusion(2047, 10.0)
    assert c.is_complex and abs(c.shift_im - 10.0 / 2048 ** 2) < 1e-20
