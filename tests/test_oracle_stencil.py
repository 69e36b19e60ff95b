"""Pins of the oracle's matrix-free stencil apply and of the backward error built on it.

``problems.apply_stencil`` evaluates A x from the stencil's definition with
shifted array slices; ``problems.assemble`` builds A as a Kronecker sum of
per-axis Toeplitz tridiagonals.  The two constructions share nothing but the
stencil description, so their agreement (to rounding) on grids with a
different coefficient on every side of every axis pins the axis order, the
side of each neighbour and the complex shift of both.  A transposed
operator, a swapped lo/hi, a dropped axis or a wrong boundary would break
it.  ``backward_error_stencil`` (the extended-precision BE on grids too large
to assemble) is pinned against the CSR-based one and against its definition
on a residual known exactly.
"""
import numpy as np
import pytest

from oracle import gadi_ref, problems

SPECS = [
    problems.convection_diffusion(2, 13, (10.0, -3.0)),
    problems.StencilSpec(2, (11, 4, 1), 4.5, (-1.25, -0.5, 0.0), (-0.75, -1.5, 0.0)),
    problems.StencilSpec(3, (7, 5, 3), 6.25, (-1.2, -0.7, -1.1), (-0.8, -1.3, -0.9)),
    problems.StencilSpec(3, (1, 6, 4), 6.0, (-1.0, -1.1, -0.6), (-1.0, -0.9, -1.4)),
    problems.complex_reaction_diffusion(9, 100.0),
]


@pytest.mark.parametrize("spec", SPECS)
def test_apply_stencil_equals_assembled_matrix(spec):
    A = problems.assemble(spec)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, spec.size)
    if spec.is_complex:
        x = x + 1j * rng.uniform(-1, 1, spec.size)
    y = problems.apply_stencil(spec, x)
    ref = A @ x
    assert y.shape == ref.shape
    scale = (abs(spec.center) + sum(map(abs, spec.lo)) + sum(map(abs, spec.hi)) + abs(spec.shift_im))
    assert np.max(np.abs(y - ref)) <= 4 * np.finfo(np.float64).eps * scale
    if spec.lo != spec.hi:
        # the transpose is a different operator on these grids: the check can tell them apart
        assert np.max(np.abs(y - A.T @ x)) > 1e-3


def test_apply_stencil_unit_vectors_give_columns():
    """A e_j is column j of A: every entry of the matrix, one basis vector at a time."""
    spec = problems.StencilSpec(3, (4, 3, 3), 6.5, (-1.2, -0.7, -1.1), (-0.8, -1.3, -0.9))
    A = problems.assemble(spec).toarray()
    for j in range(spec.size):
        e = np.zeros(spec.size)
        e[j] = 1.0
        assert np.array_equal(problems.apply_stencil(spec, e), A[:, j])


def test_apply_stencil_keeps_extended_precision():
    """In np.longdouble the products and sums carry the longer significand."""
    spec = problems.StencilSpec(2, (5, 4, 1), 4.0, (-1.0, -1.0, 0.0), (-1.0, -1.0, 0.0))
    x = np.full(spec.size, 1.0, dtype=np.longdouble) + np.longdouble(2.0) ** -60
    y = problems.apply_stencil(spec, x)
    assert y.dtype == np.longdouble
    if np.finfo(np.longdouble).nmant >= 63:
        # interior rows of the Laplacian with a constant vector: the 2^-60 parts cancel exactly
        Y = y.reshape(4, 5)
        assert np.all(Y[1:-1, 1:-1] == 0)
        assert Y[0, 0] == 2 + np.longdouble(2.0) ** -59


@pytest.mark.parametrize("spec", SPECS)
def test_backward_error_stencil_equals_csr_extended(spec):
    A = problems.assemble(spec)
    rng = np.random.default_rng(4)
    xt = rng.uniform(-1, 1, spec.size)
    x = rng.uniform(-1, 1, spec.size)
    if spec.is_complex:
        xt = xt + 1j * rng.uniform(-1, 1, spec.size)
        x = x + 1j * rng.uniform(-1, 1, spec.size)
    b = A @ xt
    for xx in (x, xt, xt + 1e-9 * x):
        ref = gadi_ref.backward_error(A, xx, b, 7.5, extended=True)
        got = gadi_ref.backward_error_stencil(spec, xx, b, 7.5)
        # the two sum in different orders in long double (about 1e-19 relative to the
        # terms); at the exact solution x_t the BE itself is only the rounding of b
        assert abs(got - ref) <= 1e-14 * ref + 1e-18


def test_backward_error_stencil_on_a_known_residual():
    """x = 0 gives BE = ||b|| / ||b|| = 1; a dyadic system gives the exact residual."""
    spec = problems.StencilSpec(2, (6, 5, 1), 4.0, (-1.0625, -0.9375, 0.0), (-0.9375, -1.0625, 0.0))
    A = problems.assemble(spec)
    xt = np.arange(spec.size, dtype=np.float64) / 8.0
    b = A @ xt                              # exact: dyadic coefficients and values
    assert gadi_ref.backward_error_stencil(spec, np.zeros(spec.size), b, 8.0) == 1.0
    assert gadi_ref.backward_error_stencil(spec, xt, b, 8.0) == 0.0
    d = np.zeros(spec.size)
    d[7] = 0.5                              # r = -A d exactly; ||A d|| from column 7
    nr = np.linalg.norm(A.toarray()[:, 7] * 0.5)
    want = nr / (8.0 * np.linalg.norm(xt + d) + np.linalg.norm(b))
    assert abs(gadi_ref.backward_error_stencil(spec, xt + d, b, 8.0) - want) <= 1e-15 * want
