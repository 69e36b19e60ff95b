"""Test-side helpers: the same workload seen by the oracle and by the HIP path.

Both sides are built from the same (dim, grid, convection) description: the
oracle assembles its CSR matrix with ``oracle.problems`` and the HIP path
gets a ``paper_2512_21164_amd.Problem``; each implements the discretization
on its own.  Inputs come from ``workloads``.
"""
import numpy as np

import workloads
from oracle import gadi_ref, problems


def oracle_system(dim, ng, beta, seed=0, dist="uniform", reaction=0.0):
    spec = problems.convection_diffusion(dim, ng, beta, reaction=reaction) if np.ndim(ng) == 0 else None
    if spec is None:
        raise ValueError("oracle_system takes a scalar grid side")
    A = problems.assemble(spec)
    x = workloads.x_true(spec.size, seed, dist)
    return spec, A, x, A @ x


def oracle_system_aniso(dim, ngs, beta, seed=0):
    """Grids with a different side per axis (h per axis), for ragged tiles."""
    ngs = tuple(ngs)
    betas = tuple(beta) if np.ndim(beta) else (beta,) * dim
    lo, hi = [], []
    for d in range(dim):
        h = 1.0 / (ngs[d] + 1)
        lo.append(-1.0 - betas[d] * h / 2)
        hi.append(-1.0 + betas[d] * h / 2)
    lo += [0.0] * (3 - dim)
    hi += [0.0] * (3 - dim)
    n = ngs + (1,) * (3 - dim)
    spec = problems.StencilSpec(dim, n, 2.0 * dim, tuple(lo), tuple(hi))
    A = problems.assemble(spec)
    x = workloads.x_true(spec.size, seed)
    return spec, A, x, A @ x


def gpu_problem(spec):
    from paper_2512_21164_amd import Problem
    return Problem(spec.dim, tuple(spec.n), spec.center, tuple(spec.lo), tuple(spec.hi),
                   shift_im=spec.shift_im, is_complex=spec.is_complex)


def to_dev(v):
    import torch
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda")


def rel(a, b):
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - b) / (den if den > 0 else 1.0))


__all__ = ["oracle_system", "oracle_system_aniso", "gpu_problem", "to_dev", "rel", "gadi_ref"]
