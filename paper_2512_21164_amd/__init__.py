"""MI355X (gfx950) implementation of mixed-precision GADI (arXiv 2512.21164).

The solver is the C-ABI library ``libgadi.so`` (include/gadi.h) built from the
HIP sources in ``csrc/``; ``api`` wraps it for PyTorch tensors, ``serve`` runs
a continuous-batching request loop on top of the batch API.
"""
from .api import (Problem, Solver, apply, autotune, autotune_class, make_params, residual, solve_noalloc,
                  workspace_bytes)

__all__ = ["Problem", "Solver", "apply", "autotune", "autotune_class", "make_params", "residual", "solve_noalloc",
           "workspace_bytes"]
