"""Problem definitions for the oracle: stencil description, assembly, splitting.

The operators are the centered finite-difference discretizations of the
paper's Section 5 (2D convection-diffusion(-reaction) in Section 5.2, 3D
convection-diffusion in Section 5.3, complex reaction-diffusion in Section
5.4), scaled by h^2 as the paper does, on the interior of a uniform grid with
homogeneous Dirichlet boundary values (h = 1/(n_g + 1)).

Readings taken where the paper leaves the discretization open:
* The convection term is discretized with the sign the PDE gives:
  for  -u'' + beta u'  the row of T_d is  lo = -1 - beta h/2 (coefficient of
  the i-1 neighbour), diag = 2, hi = -1 + beta h/2 (coefficient of i+1).
* In 3D the diagonal of A is 6 (the 7-point Laplacian after h^2 scaling).
* The complex problem  -Lap u + i sigma u  becomes  L + i sigma h^2 I  after
  scaling, and is split with the Hermitian / skew-Hermitian splitting, which is
  exactly the symmetric / skew splitting of the real block form of Section 5.4.

Unknowns are ordered x-fastest: index = i + nx * (j + ny * k).
"""
from __future__ import annotations

import dataclasses
from typing import Tuple

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass(frozen=True)
class StencilSpec:
    """A 5-point (2D) or 7-point (3D) constant-coefficient operator.

    A u at grid point i = center*u_i + sum_d (lo[d] * u_{i - e_d} + hi[d] * u_{i + e_d})
                          + 1j * shift_im * u_i      (complex problems only)
    with zero values outside the grid.
    """
    dim: int
    n: Tuple[int, int, int]          # (nx, ny, nz); nz == 1 in 2D
    center: float
    lo: Tuple[float, float, float]   # coefficient of the neighbour on the -d side
    hi: Tuple[float, float, float]   # coefficient of the neighbour on the +d side
    shift_im: float = 0.0
    is_complex: bool = False

    @property
    def size(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


def convection_diffusion(dim: int, ng: int, beta, reaction: float = 0.0) -> StencilSpec:
    """-Lap u + beta . grad u + reaction * u on the unit square / cube, times h^2.

    Section 5.2 (2D) and Section 5.3 (3D): centered differences on a uniform
    grid with spacing h = 1/(ng+1).
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    beta = tuple(float(b) for b in (beta if np.ndim(beta) else [beta] * dim))
    if len(beta) != dim:
        raise ValueError("beta needs one entry per axis")
    h = 1.0 / (ng + 1)
    lo = [-1.0 - b * h / 2.0 for b in beta] + [0.0] * (3 - dim)
    hi = [-1.0 + b * h / 2.0 for b in beta] + [0.0] * (3 - dim)
    n = (ng, ng, ng if dim == 3 else 1)
    return StencilSpec(dim, n, 2.0 * dim + reaction * h * h, tuple(lo), tuple(hi))


def complex_reaction_diffusion(ng: int, sigma: float) -> StencilSpec:
    """-Lap u + i sigma u on the unit square, times h^2 (Section 5.4, constant potential)."""
    h = 1.0 / (ng + 1)
    return StencilSpec(2, (ng, ng, 1), 4.0, (-1.0, -1.0, 0.0), (-1.0, -1.0, 0.0),
                       shift_im=sigma * h * h, is_complex=True)


def tridiag(m: int, sub: float, diag: float, sup: float) -> sp.csr_matrix:
    """m x m Toeplitz tridiagonal matrix: T[i, i-1] = sub, T[i, i] = diag, T[i, i+1] = sup."""
    rows, cols, vals = [], [], []
    for i in range(m):
        if i > 0:
            rows.append(i); cols.append(i - 1); vals.append(sub)
        rows.append(i); cols.append(i); vals.append(diag)
        if i < m - 1:
            rows.append(i); cols.append(i + 1); vals.append(sup)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, m), dtype=np.float64)


def assemble(spec: StencilSpec) -> sp.csr_matrix:
    """Assemble A as a Kronecker sum of per-axis tridiagonals (Sections 5.2, 5.3).

    With x fastest, A = I_z (x) I_y (x) T_x + I_z (x) T_y (x) I_x + T_z (x) I_y (x) I_x,
    where T_d = tridiag(lo[d], center/dim, hi[d]); the centre is split evenly
    across the axes (any split gives the same A).
    """
    nx, ny, nz = spec.n
    c = spec.center / spec.dim
    Ix, Iy, Iz = (sp.identity(m, format="csr", dtype=np.float64) for m in (nx, ny, nz))
    Tx = tridiag(nx, spec.lo[0], c, spec.hi[0])
    Ty = tridiag(ny, spec.lo[1], c, spec.hi[1])
    A = sp.kron(Iz, sp.kron(Iy, Tx)) + sp.kron(Iz, sp.kron(Ty, Ix))
    if spec.dim == 3:
        Tz = tridiag(nz, spec.lo[2], c, spec.hi[2])
        A = A + sp.kron(Tz, sp.kron(Iy, Ix))
    A = sp.csr_matrix(A)
    if spec.is_complex:
        A = sp.csr_matrix(A.astype(np.complex128) + 1j * spec.shift_im * sp.identity(spec.size))
    A.sort_indices()
    return A


def apply_stencil(spec: StencilSpec, x) -> np.ndarray:
    """y = A x straight from the stencil's definition (see ``StencilSpec``), without a matrix.

    The grid function is viewed as an array indexed (k, j, i) (x fastest) and
    each neighbour term is a shifted slice, with zero values outside the grid.
    The arithmetic is done in the dtype of x (e.g. ``np.longdouble`` for an
    extended-precision residual), which is what makes this usable on grids
    too large to assemble.
    """
    nx, ny, nz = spec.n
    X = np.asarray(x).reshape(nz, ny, nx)
    if spec.is_complex and not np.iscomplexobj(X):
        X = X.astype(np.result_type(X.dtype, np.complex64))
    Y = X * X.dtype.type(spec.center)
    if spec.is_complex:
        Y = Y + X * X.dtype.type(1j * spec.shift_im)
    for d in range(spec.dim):
        ax = 2 - d                        # axis of grid direction d in the (k, j, i) view
        n = X.shape[ax]
        if n < 2:
            continue
        head = [slice(None)] * 3
        tail = [slice(None)] * 3
        head[ax] = slice(0, n - 1)        # points that have a +d neighbour
        tail[ax] = slice(1, n)            # points that have a -d neighbour
        Y[tuple(head)] += X.dtype.type(spec.hi[d]) * X[tuple(tail)]
        Y[tuple(tail)] += X.dtype.type(spec.lo[d]) * X[tuple(head)]
    return Y.reshape(-1)


def hss_split(A: sp.spmatrix):
    """Hermitian / skew-Hermitian splitting A = M + N (eq. (split), Section 3.1).

    M = (A + A^H)/2 and N = (A - A^H)/2; for real A this is the symmetric /
    skew-symmetric splitting used in every experiment of Section 5.
    """
    AH = A.conj().T
    M = sp.csr_matrix((A + AH) * 0.5)
    N = sp.csr_matrix((A - AH) * 0.5)
    M.sort_indices(); N.sort_indices()
    return M, N


def shifted(M: sp.spmatrix, N: sp.spmatrix, alpha: float):
    """H = alpha I + M and S = alpha I + N (eq. (split), Section 3.1)."""
    I = sp.identity(M.shape[0], format="csr")
    H = sp.csr_matrix(alpha * I + M)
    S = sp.csr_matrix(alpha * I + N)
    H.sort_indices(); S.sort_indices()
    return H, S


def real_block_form(A_complex: sp.spmatrix) -> sp.csr_matrix:
    """The real 2n x 2n block form [[Re A, -Im A], [Im A, Re A]] of Section 5.4."""
    L = sp.csr_matrix(A_complex.real)
    V = sp.csr_matrix(A_complex.imag)
    return sp.csr_matrix(sp.bmat([[L, -V], [V, L]]))


def grid_function(spec: StencilSpec, f) -> np.ndarray:
    """Sample f(x1, x2[, x3]) at the interior grid points, x-fastest order."""
    nx, ny, nz = spec.n
    h = [1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1)]
    xs = (np.arange(1, nx + 1) * h[0])
    ys = (np.arange(1, ny + 1) * h[1])
    if spec.dim == 2:
        Y, X = np.meshgrid(ys, xs, indexing="ij")
        return np.asarray(f(X, Y), dtype=np.float64).ravel()
    zs = (np.arange(1, nz + 1) * h[2])
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.asarray(f(X, Y, Z), dtype=np.float64).ravel()
