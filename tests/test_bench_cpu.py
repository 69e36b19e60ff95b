"""Host logic of bench.py: the byte model of one solve and the CPU oracle sample."""
import pytest

import bench


def _hist(jh, js, sweeps=1):
    # one row per sweep [k, BE, CG iterations, CGNE iterations] and the final row
    return [[k, 0.0, jh, js] for k in range(sweeps)] + [[sweeps, 0.0, 0, 0]]


@pytest.mark.parametrize("s,cplx,dim,ry,paired", [
    (8, False, 3, 4, True), (4, False, 2, 1, True), (4, False, 3, 1, True),
    (8, True, 2, 1, True), (4, True, 2, 1, True), (4, True, 3, 1, False),
    (2, False, 2, 1, False), (2, False, 3, 1, False), (2, False, 3, 2, True), (2, False, 3, 4, True),
    (2, True, 2, 1, False),
])
def test_pairing_classes(s, cplx, dim, ry, paired):
    """The default pairing follows the kernel classes that update z every second CG iteration."""
    h = _hist(8, 2)
    default = bench.alg_bytes(h, 1, s, cplx=cplx, dim=dim, ry=ry)
    assert default == bench.alg_bytes(h, 1, s, cplx=cplx, pair_z=paired)


@pytest.mark.parametrize("s", [2, 4, 8])
@pytest.mark.parametrize("m", [2, 3, 5, 10])
def test_pairing_saves_s_per_two_iterations(s, m):
    """An even CG count 2m >= 4 moves (m - 2) s fewer bytes per unknown with the paired z update
    (one z read-write per two iterations, plus the older direction and the fold)."""
    h = _hist(2 * m, 3)
    plain = bench.alg_bytes(h, 1, s, pair_z=False)
    paired = bench.alg_bytes(h, 1, s, pair_z=True)
    assert plain - paired == (m - 2) * s


def test_odd_count_has_no_fold():
    """With an odd CG count the last pending term is the usual single one: no fold pass."""
    s = 4
    odd = bench.alg_bytes(_hist(5, 0), 1, s, pair_z=True)
    even = bench.alg_bytes(_hist(4, 0), 1, s, pair_z=True)
    # iteration j = 4 (first pass 6s, second 3s) against the fold after 4 iterations (3s)
    assert odd - even == 6 * s + 3 * s - 3 * s


def test_bytes_scale_with_unknowns_and_complex_has_no_cgne():
    h = _hist(6, 2, sweeps=3)
    assert bench.alg_bytes(h, 1000, 4) == 1000 * bench.alg_bytes(h, 1, 4)
    # complex problems solve S pointwise inside the outer phase: CGNE counts move no bytes
    assert bench.alg_bytes(_hist(6, 5, 2), 1, 4, cplx=True) == bench.alg_bytes(_hist(6, 0, 2), 1, 4, cplx=True)


def test_method_bytes_per_unit():
    """The method's per-unit figures: 24 + 2s per sweep, 10s per CG or CGNE iteration."""
    assert bench.alg_bytes_unit(3, 10, 4, 1, 4) == 3 * 32 + 14 * 40
    assert bench.alg_bytes_unit(3, 10, 4, 1, 4, cplx=True) == 2 * (3 * 32 + 14 * 40)


def test_cpu_oracle_sample_is_sized_and_described():
    """The oracle sample runs at least one timed sweep, scales by the unknown count and says so."""
    r = bench.cpu_baseline(2, 64, 32, 1.0, 0.5, 4, 2, 0, "f64", 100, 8.0, seconds=0.2)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "solves/s"
    assert r["value"] > 0 and r["scaled"] is True
    assert "sweep" in r["sample"] and "32x32" in r["sample"] and "(4x)" in r["sample"]
    r = bench.cpu_baseline(2, 32, 32, 1.0, 0.5, 4, 2, 3, "f32", 100, 8.0)
    assert r["scaled"] is False and r["sample"].startswith("3 GADI sweep(s)")
