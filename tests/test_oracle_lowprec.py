"""Pins of the oracle's low-precision emulation and of mixed-precision behaviour.

* BF16 rounding is checked against a brute-force nearest search over every
  finite BF16 value, and against Table 1's unit roundoff (golden file).
* Theorem 3 and the simplified rates of Section 3.4 predict that inner solves
  in FP32 or BF16 leave the backward-error limit at O(u) and barely change the
  number of outer sweeps while c(n) kappa(H) kappa(S) u_s << rho(T_F).
"""
import os

import numpy as np
import pytest

import workloads
from oracle import gadi_ref, lowprec, problems

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "unit_roundoff_table1.txt")


def _table1():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, bits, u = line.split()
        out[name] = (int(bits), float(u))
    return out


def _all_bf16_values():
    bits = (np.arange(0, 1 << 16, dtype=np.uint32) << 16).view(np.float32)
    vals = bits[np.isfinite(bits)]
    return np.unique(vals.astype(np.float64))


def _brute_nearest_bf16(x, table):
    """Nearest BF16 value by search; ties go to the value with an even last bit."""
    out = np.empty_like(x)
    for i, v in enumerate(x.astype(np.float64)):
        k = np.searchsorted(table, v)
        cands = [table[j] for j in (k - 1, k) if 0 <= j < len(table)]
        d = [abs(c - v) for c in cands]
        best = min(d)
        ties = [c for c, dd in zip(cands, d) if dd == best]
        if len(ties) == 1:
            out[i] = ties[0]
        else:
            even = [c for c in ties if (np.float32(c).view(np.uint32) >> 16) & 1 == 0]
            out[i] = even[0]
    return out


def test_bf16_rounding_matches_brute_force_nearest():
    rng = np.random.default_rng(11)
    table = _all_bf16_values()
    x = (rng.standard_normal(3000) * 10.0 ** rng.uniform(-30, 30, 3000)).astype(np.float32)
    # exact ties: midpoints between neighbouring BF16 values
    lo = (rng.integers(1, 0x7F00, 500).astype(np.uint32) << 16)
    mid = (lo | np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, mid, -mid, np.float32([0.0, -0.0, 1.0, 3.0e38])])
    got = lowprec.round_bf16(x).astype(np.float64)
    want = _brute_nearest_bf16(x, table)
    assert np.array_equal(got, want)


def test_bf16_rounding_agrees_with_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    x = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-20, 20, 100000)).astype(np.float32)
    t = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(lowprec.round_bf16(x), t)


def test_unit_roundoffs_match_table1():
    tab = _table1()
    for name, key in (("bf16", "bf16"), ("fp32", "f32"), ("fp64", "f64")):
        bits, u_printed = tab[name]
        u = lowprec.UNIT_ROUNDOFF[key]
        assert u == 2.0 ** -bits
        assert float(f"{u:.2e}") == u_printed
    rng = np.random.default_rng(13)
    x = rng.uniform(-1e6, 1e6, 200000).astype(np.float32)
    rel = np.abs(lowprec.round_bf16(x).astype(np.float64) - x) / np.abs(x)
    assert rel.max() <= tab["bf16"][1] * 1.001
    assert rel.max() > 0.5 * tab["bf16"][1]
    y = rng.uniform(-1e6, 1e6, 200000)
    rel32 = np.abs(y.astype(np.float32).astype(np.float64) - y) / np.abs(y)
    assert rel32.max() <= tab["fp32"][1] * 1.001


def _system(ng=32, beta=(10.0, 10.0), seed=0):
    spec = problems.convection_diffusion(2, ng, beta)
    A = problems.assemble(spec)
    x = workloads.x_true(spec.size, seed)
    return spec, A, x, A @ x, gadi_ref.norm2(A)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_precision_reaches_fp64_backward_error(prec):
    """Theorem 3: the backward-error limit is O(u), not O(u_s)."""
    spec, A, x, b, nA = _system()
    res = gadi_ref.gadi(A, b, 0.3, 1.0, normA=nA, tol=1e-14, max_outer=3000, prec=prec)
    assert res.status == gadi_ref.OK
    assert gadi_ref.backward_error(A, res.x, b, nA, extended=True) <= 1.5e-14


def test_outer_count_nearly_independent_of_inner_precision():
    """Section 3.4: rates depend on u_s only through c(n) kappa(H) kappa(S) u_s."""
    spec, A, x, b, nA = _system(ng=24, beta=(1.0, 1.0))
    outs = {}
    for prec in ("f64", "f32", "bf16"):
        res = gadi_ref.gadi(A, b, 0.5, 1.0, normA=nA, tol=1e-10, max_outer=5000, prec=prec)
        assert res.status == gadi_ref.OK
        outs[prec] = res.outer
    for prec in ("f32", "bf16"):
        assert abs(outs[prec] - outs["f64"]) <= 0.03 * outs["f64"] + 2

