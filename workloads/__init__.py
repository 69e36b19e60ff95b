"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the GADI method: it only draws random
numbers and describes workloads (grid sizes, convection coefficients, the
alpha sweep, arrival traces).  Both the CPU oracle and the product path take
their inputs from here, so that the two sides see bit-identical data.

Workloads follow the experiments of the paper's Section 5 (convection-
diffusion in 2D and 3D, complex reaction-diffusion), restated as synthetic
systems: the right-hand side is either b = A x_true with a seeded x_true, or
a seeded random vector.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np


def x_true(n: int, seed: int = 0, dist: str = "uniform") -> np.ndarray:
    """Seeded exact solution, float64 of length n.

    dist="uniform": U(-1, 1); dist="normal": N(0, 1).
    """
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=n).astype(np.float64)
    if dist == "normal":
        return rng.standard_normal(size=n).astype(np.float64)
    raise ValueError(f"unknown distribution {dist!r}")


def dyadic_field(n, bits: int = 24, seed: int = 0) -> np.ndarray:
    """Smooth seeded grid function with few significant bits, x-fastest.

    n = (nx, ny, nz): a seeded amplitude in [0.5, 1] times the product over
    the axes of length > 1 of sin(pi t_d) (t_d the interior grid coordinates):
    the smoothest mode, for which ||b|| = ||A x|| is smallest against
    ||A|| ||x||, rounded to a multiple of 2^-bits.  With dyadic stencil coefficients, A applied to it is exactly
    representable in float64, so b = A x is exact and x is the exact solution
    of the float64 system.
    """
    rng = np.random.default_rng(seed)
    f = np.full(1, rng.uniform(0.5, 1.0))
    for m in n:
        t = np.arange(1, m + 1) / (m + 1)
        f = np.multiply.outer(np.sin(np.pi * t) if m > 1 else np.ones(1), f)
    return np.round(f.ravel() * 2.0 ** bits) / 2.0 ** bits


def perturbation(n: int, scale: float, seed: int = 0) -> np.ndarray:
    """Seeded float64 vector with entries scale * U(-1, 1)."""
    rng = np.random.default_rng(seed)
    return scale * rng.uniform(-1.0, 1.0, size=n)


def complex_rhs(n: int, seed: int = 0) -> np.ndarray:
    """Seeded complex right-hand side, real and imaginary parts ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=n)
    im = rng.uniform(-1.0, 1.0, size=n)
    return (re + 1j * im).astype(np.complex128)


def alpha_sweep(count: int = 8, lo_exp: float = -3.0, hi_exp: float = 0.0) -> np.ndarray:
    """Log-spaced regularization parameters, 1e-3 .. 1 by default."""
    return np.logspace(lo_exp, hi_exp, count)


@dataclasses.dataclass(frozen=True)
class Request:
    """One solve request of the serving workload."""
    rid: int
    arrival_s: float      # arrival time from the start of the trace
    dim: int              # 2 or 3
    side: int             # interior points per axis
    beta: float           # convection coefficient on every axis
    alpha: float          # regularization parameter
    seed: int             # seed of x_true for this request

    @property
    def n(self) -> int:
        return self.side ** self.dim


def poisson_trace(num: int = 512, rate_per_s: float = 200.0, seed: int = 0,
                  side2d=(32, 1024), side3d=(16, 128), beta_max: float = 50.0,
                  alpha_exp=(-3.0, 0.0)) -> List[Request]:
    """Poisson arrival trace of convection-diffusion solve requests.

    Inter-arrival gaps are exponential with mean 1/rate.  Each request is 2D
    with probability 1/2 (side uniform in side2d) else 3D (side uniform in
    side3d); beta ~ U(0, beta_max); alpha = 10**U(alpha_exp).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=num)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(num):
        r = np.random.default_rng(1000 + i)
        dim = 2 if r.uniform() < 0.5 else 3
        lo, hi = side2d if dim == 2 else side3d
        side = int(r.integers(lo, hi + 1))
        beta = float(r.uniform(0.0, beta_max))
        alpha = float(10.0 ** r.uniform(*alpha_exp))
        out.append(Request(i, float(t[i]), dim, side, beta, alpha, 1000 + i))
    return out


def scale_trace(trace: List[Request], max_side2d: int, max_side3d: int) -> List[Request]:
    """Clamp request sides (for reduced-size rehearsals of the serving workload)."""
    out = []
    for q in trace:
        cap = max_side2d if q.dim == 2 else max_side3d
        out.append(dataclasses.replace(q, side=min(q.side, cap)))
    return out


__all__ = ["x_true", "complex_rhs", "alpha_sweep", "Request", "poisson_trace",
           "scale_trace"]
