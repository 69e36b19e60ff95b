"""Storage rounding for the emulated low precision u_s (oracle only).

Table 1 of the paper lists the formats; its unit roundoffs (BF16 2^-8,
FP32 2^-24) assume round-to-nearest.  The casts in Algorithm 1 (the FP64
residual to u_s, Lemma 2 in Section 3.2) are taken as round-to-nearest-even.

``round_bf16`` rounds float32 values to the nearest bfloat16 value (8
significand bits), ties to even, and returns them as float32.  It follows the
definition: keep the upper 16 bits of the float32 encoding, and add one unit
in the last kept place when the dropped 16 bits exceed half a unit, or equal
half a unit while the kept part is odd.  NaNs stay NaN.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x) -> np.ndarray:
    """Round float32 (or complex64, per component) values to BF16, ties to even."""
    a = np.asarray(x)
    if np.iscomplexobj(a):
        a = a.astype(np.complex64)
        return (round_bf16(a.real) + 1j * round_bf16(a.imag)).astype(np.complex64)
    a = np.ascontiguousarray(a, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    kept = bits >> 16                     # sign, exponent, 7 stored significand bits
    dropped = bits & 0xFFFF               # the 16 bits that do not fit
    half = 0x8000
    round_up = (dropped > half) | ((dropped == half) & ((kept & 1) == 1))
    kept = kept + round_up.astype(np.uint64)
    out = (kept << 16).astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    if nan.any():
        out = out.copy()
        out[nan] = np.float32("nan")
    return out.reshape(np.shape(x))


PRECISIONS = ("f64", "f32", "bf16")


def arith_dtype(prec: str, is_complex: bool):
    """Arithmetic dtype of the inner solves for precision ``prec``.

    BF16 storage is paired with FP32 arithmetic (Section 5.1, BF16 variant).
    """
    if prec == "f64":
        return np.complex128 if is_complex else np.float64
    if prec in ("f32", "bf16"):
        return np.complex64 if is_complex else np.float32
    raise ValueError(f"unknown precision {prec!r}")


def store(v, prec: str):
    """Round a vector to the storage format of precision ``prec``."""
    if prec == "bf16":
        return round_bf16(v)
    return np.asarray(v, dtype=arith_dtype(prec, np.iscomplexobj(v)))


UNIT_ROUNDOFF = {"bf16": 2.0 ** -8, "f32": 2.0 ** -24, "f64": 2.0 ** -53}
