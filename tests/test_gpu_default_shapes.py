"""The library's default tile shapes (no tile_ry / tile_chunk given, no tuned entry).

3D rows per wave follow the grid size: one row below 2^24 unknowns (FP32 and
FP64 inner solves) or 2^26 (BF16), four or two rows from there on, one row for
complex problems.  2D BF16 tilings take twice the one-round chunk when at least
half the resident waves still get a tile.  Handles are created with a given
||A|| (no norm estimate) and never solve, so the large grids cost only their
workspace.
"""
import pytest

pytestmark = pytest.mark.gpu


def _tiling(dim, n, u_s, **kw):
    from paper_2512_21164_amd import Problem, Solver
    pr = Problem.convection_diffusion(dim, n, 10.0)     # n: a side or a per-axis tuple
    s = Solver(pr, alpha=0.05, u_s=u_s, normA=12.0, **kw)
    t = s.tiling
    s.close()
    return t


@pytest.mark.parametrize("n,u_s,ry", [
    (64, "f32", 1), ((256, 256, 255), "f32", 1), (256, "f32", 4),
    ((256, 256, 255), "f64", 1), (256, "f64", 4),
    (256, "bf16", 1), ((512, 512, 255), "bf16", 1), ((512, 512, 256), "bf16", 2),
])
def test_3d_rows_per_wave_by_size(gpu_lib, n, u_s, ry):
    assert _tiling(3, n, u_s)["ry"] == ry


def test_3d_explicit_rows_override_the_default(gpu_lib):
    assert _tiling(3, 64, "f32", tile_ry=4)["ry"] == 4
    assert _tiling(3, 256, "f32", tile_ry=1)["ry"] == 1


def test_2d_bf16_chunk(gpu_lib):
    # tile_chunk = -1: one-round chunks (share factor 1) without the BF16 rule
    big, big1 = _tiling(2, 4096, "bf16"), _tiling(2, 4096, "bf16", tile_chunk=-1)
    assert big["chunk_inner"] == 2 * big1["chunk_inner"]
    small, small1 = _tiling(2, 1024, "bf16"), _tiling(2, 1024, "bf16", tile_chunk=-1)
    assert small["chunk_inner"] == small1["chunk_inner"]
    f32, f32_1 = _tiling(2, 4096, "f32"), _tiling(2, 4096, "f32", tile_chunk=-1)
    assert f32["chunk_inner"] == f32_1["chunk_inner"]
