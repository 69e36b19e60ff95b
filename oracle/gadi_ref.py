"""Reference GADI iteration (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Algorithm 1 of Section 2.3 (mixed-precision GADI), run step by step:

    x^(0) = 0
    repeat
        r^(k) = b - A x^(k)                              (u_r = FP64, or exact)
        solve (alpha I + M) z^(k) = r^(k)                (u_s)
        solve (alpha I + N) y^(k) = (2 - omega) alpha z^(k)   (u_s)
        x^(k+1) = x^(k) + y^(k)                          (u = FP64)
    until convergence

Inner solvers (Section 5.1): conjugate gradients on H = alpha I + M, and CG
on the normal equations for S = alpha I + N.  The normal-equation variant is
read as Craig's method (CGNE), whose recursive residual is the residual of
S y = c itself.  Both start from a zero guess and stop on the relative
residual ||r_j|| <= tol ||r_0||, at a cap, or on stagnation (Section 5.1,
early stop for BF16).

Inner precision u_s is emulated: "f64" uses float64, "f32" float32 storage
and arithmetic, "bf16" BF16 storage (round-to-nearest-even after every
vector update) with float32 arithmetic; the operator coefficients are held in
the arithmetic format (float32 for f32 and bf16).

Stopping and status rules of the outer loop (readings of Sections 3, 4.3 and 5.1):
at the top of sweep k the residual of x^(k) is formed and
    BE_k = ||r|| / (||A|| ||x^(k)|| + ||b||)           (backward error, Section 3)
    relres_k = ||r|| / ||r^(0)||                        (the paper's Section 5 test)
The iteration returns x^(k) with status
    OK            when the chosen criterion <= tol,
    DIVERGED      when BE_k is not finite or exceeds div_factor * min_j BE_j,
    STAGNATED     when BE has not dropped below 0.99 of its last reference
                  value for stag_window sweeps,
    NOT_CONVERGED when k == max_outer,
checked in that order.

Residual precision u_r (Section 2.3): "f64" forms b - A x in float64; "exact"
is the extra-precision residual taken to its limit, b - A x computed exactly
and rounded once to float64 (``residual_exact``).

Alpha selection (Section 4.3): ``safeguarded_alpha`` raises alpha by a fixed
factor until kappa(H) kappa(S) u_s < tau (closed-form condition numbers), and
``gadi_select_alpha`` restarts with a larger alpha after an attempt that
stagnated or diverged (from the last iterate, or from zero after divergence),
all attempts sharing one sweep budget.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import lowprec
from .problems import hss_split, shifted

OK, NOT_CONVERGED, STAGNATED, DIVERGED = 0, 1, 2, 3
STATUS_NAMES = {OK: "OK", NOT_CONVERGED: "NOT_CONVERGED", STAGNATED: "STAGNATED",
                DIVERGED: "DIVERGED"}

# ||r_j|| must fall below 0.99 * (best so far) to count as progress: in
# squared norms that is a factor 0.99**2.
PROGRESS_SQ = 0.9801
PROGRESS = 0.99


@dataclasses.dataclass
class InnerRule:
    """Stopping rule of one inner solve (Section 5.1)."""
    tol: float = 1e-3          # relative residual tolerance
    max_iter: int = 2000       # cap on iterations
    fixed: int = 0             # > 0: run exactly this many iterations, ignore the rest
    stag_window: int = 20      # early stop: no 1% progress in this many iterations (0: off)

    def stop(self, it: int, rho_new: float, rho0: float, tracker) -> bool:
        """Decide after iteration ``it`` (1-based) with squared residual norm rho_new."""
        if self.fixed > 0:
            return it >= self.fixed
        if not np.isfinite(rho_new):
            return True
        if rho_new <= (self.tol * self.tol) * rho0:
            return True
        if it >= self.max_iter:
            return True
        if rho_new < PROGRESS_SQ * tracker[0]:
            tracker[0] = rho_new
            tracker[1] = it
        if self.stag_window > 0 and it - tracker[1] >= self.stag_window:
            return True
        return False


def _rdot(a, b) -> float:
    """Real part of a^H b in the arithmetic precision of the inputs."""
    return np.real(np.vdot(a, b))


def cg(H, c, rule: InnerRule, prec: str = "f64"):
    """Conjugate gradients on the Hermitian positive definite H, zero initial guess.

    Returns (z, iterations).  Each iteration: q = H p; a = rho / (p, q);
    z += a p; r -= a q; rho' = (r, r); beta = rho'/rho; p = r + beta p.
    """
    cplx = np.iscomplexobj(c) or np.iscomplexobj(H.data)
    dt = lowprec.arith_dtype(prec, cplx)
    rt = np.float64 if prec == "f64" else np.float32
    Hs = sp.csr_matrix(H, dtype=dt)
    r = lowprec.store(np.asarray(c, dtype=dt), prec)
    z = np.zeros_like(r)
    rho0 = rt(_rdot(r, r))
    if rho0 == 0:
        return z, 0
    p = r.copy()
    rho = rho0
    tracker = [float(rho0), 0]
    it = 0
    with np.errstate(all="ignore"):
        while True:
            q = Hs @ p
            a = rt(rho / rt(_rdot(p, q)))
            z = lowprec.store(z + a * p, prec)
            r = lowprec.store(r - a * q, prec)
            rho_new = rt(_rdot(r, r))
            it += 1
            if rule.stop(it, float(rho_new), float(rho0), tracker):
                return z, it
            beta = rt(rho_new / rho)
            p = lowprec.store(r + beta * p, prec)
            rho = rho_new


def cgne(S, c, rule: InnerRule, prec: str = "f64"):
    """Craig's method (CG on S S^H w = c, y = S^H w), zero initial guess.

    Returns (y, iterations).  Each iteration: a = rho / (p, p); y += a p;
    r -= a S p; rho' = (r, r); beta = rho'/rho; p = S^H r + beta p, with
    p_0 = S^H c.  The recursive residual r_j is the residual c - S y_j.
    """
    cplx = np.iscomplexobj(c) or np.iscomplexobj(S.data)
    dt = lowprec.arith_dtype(prec, cplx)
    rt = np.float64 if prec == "f64" else np.float32
    Ss = sp.csr_matrix(S, dtype=dt)
    SHs = sp.csr_matrix(S.conj().T, dtype=dt)
    r = lowprec.store(np.asarray(c, dtype=dt), prec)
    y = np.zeros_like(r)
    rho0 = rt(_rdot(r, r))
    if rho0 == 0:
        return y, 0
    p = lowprec.store(SHs @ r, prec)
    rho = rho0
    tracker = [float(rho0), 0]
    it = 0
    with np.errstate(all="ignore"):
        while True:
            a = rt(rho / rt(_rdot(p, p)))
            y = lowprec.store(y + a * p, prec)
            r = lowprec.store(r - a * (Ss @ p), prec)
            rho_new = rt(_rdot(r, r))
            it += 1
            if rule.stop(it, float(rho_new), float(rho0), tracker):
                return y, it
            beta = rt(rho_new / rho)
            p = lowprec.store(SHs @ r + beta * p, prec)
            rho = rho_new


def _be(nr, denom):
    """||r|| / (||A|| ||x|| + ||b||), and 0 for an exact residual: the backward error is the
    smallest relative perturbation of A and b that x solves exactly (Section 3), which is zero
    when r = 0, also where the quotient is 0 / 0 (b = 0 and x = 0)."""
    return 0.0 if nr == 0 else float(nr / denom)


def backward_error(A, x, b, normA: float, extended: bool = False) -> float:
    """Normwise backward error ||b - A x|| / (||A|| ||x|| + ||b||), 2-norms (Section 3).

    With extended=True the residual is accumulated in np.longdouble.
    """
    if extended:
        cplx = np.iscomplexobj(A.data) or np.iscomplexobj(x) or np.iscomplexobj(b)
        dt = np.clongdouble if cplx else np.longdouble
        xl = np.asarray(x, dtype=dt)
        bl = np.asarray(b, dtype=dt)
        r = bl - sp.csr_matrix(A).astype(dt) @ xl
        nr = np.sqrt(np.sum(np.abs(r) ** 2))
        nx = np.sqrt(np.sum(np.abs(xl) ** 2))
        nb = np.sqrt(np.sum(np.abs(bl) ** 2))
        return _be(nr, np.longdouble(normA) * nx + nb)
    r = b - A @ x
    return _be(np.linalg.norm(r), normA * np.linalg.norm(x) + np.linalg.norm(b))


def backward_error_stencil(spec, x, b, normA: float) -> float:
    """The backward error of Section 3 with the residual b - A x accumulated in
    ``np.longdouble`` from the stencil's definition (``problems.apply_stencil``):
    for grids too large to assemble A."""
    from .problems import apply_stencil
    cplx = spec.is_complex or np.iscomplexobj(x) or np.iscomplexobj(b)
    dt = np.clongdouble if cplx else np.longdouble
    xl = np.asarray(x).astype(dt)
    r = np.asarray(b).astype(dt)
    r -= apply_stencil(spec, xl)
    nr = np.sqrt(np.sum(np.abs(r) ** 2))
    del r
    nx = np.sqrt(np.sum(np.abs(xl) ** 2))
    nb = np.sqrt(np.sum(np.abs(np.asarray(b).astype(dt)) ** 2))
    return _be(nr, np.longdouble(normA) * nx + nb)


def _split(v):
    """Veltkamp's splitting: v = hi + lo exactly, each half with at most 26
    significant bits (float64, factor 2^27 + 1; no overflow for |v| < 1e300)."""
    c = 134217729.0 * v
    hi = c - (c - v)
    return hi, v - hi


def _exact_products(a, v):
    """The four float64 products of the halves of a and v; they sum to a*v exactly
    (26 x 26 bits fit the 53-bit significand; no underflow for the magnitudes
    used here)."""
    ah, al = _split(np.asarray(a, dtype=np.float64))
    vh, vl = _split(np.asarray(v, dtype=np.float64))
    return np.stack([ah * vh, ah * vl, al * vh, al * vl], axis=-1)


def residual_exact(A, b, x) -> np.ndarray:
    """r = b - A x computed exactly and rounded once to float64 per entry.

    This is the residual in extra precision u_r (Section 2.3) in its limit
    u_r -> 0.  Each product a_ij x_j is expanded into exact float64 pieces and
    ``math.fsum`` (Shewchuk's exact summation) returns the correctly rounded
    sum of b_i and the negated pieces.  Complex entries are expanded into their
    real products.
    """
    A = sp.csr_matrix(A)
    cplx = np.iscomplexobj(A.data) or np.iscomplexobj(x) or np.iscomplexobj(b)
    n = A.shape[0]
    xv = np.asarray(x)[A.indices]
    ptr = A.indptr
    if not cplx:
        P = -_exact_products(A.data.real, xv.real)
        bb = np.asarray(b, dtype=np.float64)
        return np.array([math.fsum([bb[i], *P[ptr[i]:ptr[i + 1]].ravel()]) for i in range(n)])
    a = A.data.astype(np.complex128)
    xv = xv.astype(np.complex128)
    # (a x).re = a.re x.re - a.im x.im,  (a x).im = a.re x.im + a.im x.re
    Pre = np.concatenate([-_exact_products(a.real, xv.real), _exact_products(a.imag, xv.imag)], axis=1)
    Pim = np.concatenate([-_exact_products(a.real, xv.imag), -_exact_products(a.imag, xv.real)], axis=1)
    bb = np.asarray(b, dtype=np.complex128)
    re = [math.fsum([bb[i].real, *Pre[ptr[i]:ptr[i + 1]].ravel()]) for i in range(n)]
    im = [math.fsum([bb[i].imag, *Pim[ptr[i]:ptr[i + 1]].ravel()]) for i in range(n)]
    return np.array(re) + 1j * np.array(im)


def residual(A, b, x, u_r: str = "f64") -> np.ndarray:
    """The residual step of Algorithm 1 in precision u_r: "f64" or "exact"."""
    if u_r == "f64":
        return b - A @ x
    if u_r == "exact":
        return residual_exact(A, b, x)
    raise ValueError("u_r must be 'f64' or 'exact'")


def forward_error(x, x_ref) -> float:
    """||x - x_ref|| / ||x_ref|| (Section 3)."""
    return float(np.linalg.norm(np.asarray(x) - np.asarray(x_ref)) / np.linalg.norm(x_ref))


def norm2(A) -> float:
    """||A||_2: dense SVD for small A, else the largest singular value from ARPACK."""
    n = A.shape[0]
    if n <= 1024:
        return float(np.linalg.norm(A.toarray(), 2))
    s = spla.svds(sp.csr_matrix(A), k=1, return_singular_vectors=False, tol=1e-14)
    return float(s[0])


@dataclasses.dataclass
class GadiResult:
    x: np.ndarray
    status: int
    outer: int
    be: List[float]
    relres: List[float]
    inner_h: List[int]
    inner_s: List[int]
    iterates: Optional[List[np.ndarray]] = None

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


def gadi(A, b, alpha: float, omega: float, *, normA: float, tol: float = 1e-10,
         stop: str = "be", max_outer: int = 10000, inner: str = "mirror",
         prec: str = "f64", rule_h: Optional[InnerRule] = None,
         rule_s: Optional[InnerRule] = None, x0=None, stag_window: int = 200,
         div_factor: float = 1e3, record_iterates: bool = False, u_r: str = "f64") -> GadiResult:
    """Run Algorithm 1 (Section 2.3) on A x = b with the HSS splitting.

    u_r = "f64" or "exact" selects the precision of the residual step.

    inner = "mirror": CG on H and Craig CGNE on S in precision ``prec``.
    inner = "exact":  direct sparse LU solves of H and S (float64/complex128).
    """
    if not alpha > 0:
        raise ValueError("alpha must be > 0")
    if not 0.0 <= omega < 2.0:
        raise ValueError("omega must lie in [0, 2)")
    rule_h = rule_h or InnerRule()
    rule_s = rule_s or InnerRule()
    A = sp.csr_matrix(A)
    cplx = np.iscomplexobj(A.data) or np.iscomplexobj(b)
    wt = np.complex128 if cplx else np.float64
    b = np.asarray(b, dtype=wt)
    M, N = hss_split(A)
    H, S = shifted(M, N, alpha)
    gamma = (2.0 - omega) * alpha
    if inner == "exact":
        luH = spla.splu(sp.csc_matrix(H, dtype=wt))
        luS = spla.splu(sp.csc_matrix(S, dtype=wt))
    x = np.zeros(A.shape[0], dtype=wt) if x0 is None else np.array(x0, dtype=wt)
    normb = float(np.linalg.norm(b))
    res = GadiResult(x, OK, 0, [], [], [], [], [] if record_iterates else None)
    be_best = np.inf
    be_ref, k_ref = np.inf, 0
    nr0 = None
    k = 0
    with np.errstate(all="ignore"):
        while True:
            if record_iterates:
                res.iterates.append(x.copy())
            r = residual(A, b, x, u_r)                       # residual in u_r
            nr = float(np.linalg.norm(r))
            be = _be(nr, normA * float(np.linalg.norm(x)) + normb)
            if nr0 is None:
                nr0 = nr
            relres = nr / nr0 if nr0 > 0 else 0.0
            res.be.append(be)
            res.relres.append(relres)
            crit = be if stop == "be" else relres
            if crit <= tol:
                res.status = OK
                break
            if not np.isfinite(be) or (div_factor > 0 and be > div_factor * be_best):
                res.status = DIVERGED
                break
            be_best = min(be_best, be)
            if k == 0 or be < PROGRESS * be_ref:
                be_ref, k_ref = be, k
            if stag_window > 0 and k - k_ref >= stag_window:
                res.status = STAGNATED
                break
            if k >= max_outer:
                res.status = NOT_CONVERGED
                break
            if inner == "exact":
                z = luH.solve(r)
                y = luS.solve(gamma * z)
                jh = js = 1
            else:
                rs = lowprec.store(r.astype(lowprec.arith_dtype(prec, cplx)), prec)  # cast to u_s
                z, jh = cg(H, rs, rule_h, prec)
                c = lowprec.store(gamma * z, prec)
                y, js = cgne(S, c, rule_s, prec)
            res.inner_h.append(jh)
            res.inner_s.append(js)
            x = x + np.asarray(y, dtype=wt)                  # update in u = FP64
            k += 1
    res.x = x
    res.outer = k
    return res


def gadi_two_step(A, b, alpha: float, omega: float, sweeps: int, x0=None):
    """The two-step GADI form of Section 2.1 with exact solves, ``sweeps`` times.

    (alpha I + M) x^(k+1/2) = (alpha I - N) x^(k) + b
    (alpha I + N) x^(k+1)   = (N - (1 - omega) alpha I) x^(k) + (2 - omega) alpha x^(k+1/2)
    Returns the list of iterates x^(0..sweeps).
    """
    A = sp.csr_matrix(A)
    wt = np.complex128 if np.iscomplexobj(A.data) or np.iscomplexobj(b) else np.float64
    M, N = hss_split(A)
    I = sp.identity(A.shape[0], format="csr")
    luH = spla.splu(sp.csc_matrix(alpha * I + M, dtype=wt))
    luS = spla.splu(sp.csc_matrix(alpha * I + N, dtype=wt))
    x = np.zeros(A.shape[0], dtype=wt) if x0 is None else np.array(x0, dtype=wt)
    out = [x.copy()]
    for _ in range(sweeps):
        xh = luH.solve((alpha * I - N) @ x + b)
        x = luS.solve((N - (1.0 - omega) * alpha * I) @ x + (2.0 - omega) * alpha * xh)
        out.append(x.copy())
    return out


# --------------------------------------------------------------------------
# Alpha selection and restarts (Section 4.3, steps 2 and 3)
# --------------------------------------------------------------------------
ALPHA_GROWTH = 10.0 ** (3.0 / 7.0)   # one step of eight log-spaced values of [1e-3, 1]


def safeguarded_alpha(spec, alpha: float, prec: str, tau: float, growth: float = ALPHA_GROWTH) -> float:
    """Step 2: the smallest alpha * growth^m (m >= 0) with kappa(H) kappa(S) u_s < tau.

    kappa(H) and kappa(S) are the closed forms of ``closed_forms`` (exact for H;
    for the normal S an upper bound, exact when N has a zero eigenvalue);
    u_s is the unit roundoff of Table 1.  tau <= 0 disables the check.
    """
    from . import closed_forms
    if tau <= 0.0:
        return float(alpha)
    u = lowprec.UNIT_ROUNDOFF[prec]
    if not tau > u:
        raise ValueError("tau must exceed the unit roundoff of u_s")
    a = float(alpha)
    for _ in range(4097):
        if closed_forms.kappa_H(spec, a) * closed_forms.kappa_S(spec, a) * u < tau:
            return a
        a *= growth
    raise ValueError("alpha safeguard cannot be met")


@dataclasses.dataclass
class RestartResult:
    x: np.ndarray
    status: int
    outer: int              # sweeps over all attempts
    inner_h: int            # CG iterations over all attempts
    inner_s: int
    alpha: float            # alpha of the last attempt
    restarts: int
    attempts: List[GadiResult]

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


def gadi_select_alpha(A, b, alpha: float, omega: float, *, spec, normA: float, tau: float = 0.0,
                      growth: float = ALPHA_GROWTH, max_restarts: int = 0, max_outer: int = 10000,
                      prec: str = "f64", x0=None, **kw) -> RestartResult:
    """Section 4.3: start from the safeguarded alpha (step 2); when an attempt ends
    STAGNATED or DIVERGED, stop, multiply alpha by ``growth`` and run again (step 3)
    from the last iterate (stagnation) or from zero (divergence), while restarts
    and sweeps of the shared ``max_outer`` budget remain."""
    a = safeguarded_alpha(spec, alpha, prec, tau, growth)
    n = A.shape[0]
    cplx = np.iscomplexobj(A.data) if hasattr(A, "data") else False
    cplx = cplx or np.iscomplexobj(b)
    wt = np.complex128 if cplx else np.float64
    x = np.zeros(n, dtype=wt) if x0 is None else np.array(x0, dtype=wt)
    used, restarts, attempts = 0, 0, []
    while True:
        res = gadi(A, b, a, omega, normA=normA, max_outer=max_outer - used, prec=prec, x0=x, **kw)
        attempts.append(res)
        used += res.outer
        if res.status in (STAGNATED, DIVERGED) and restarts < max_restarts and used < max_outer:
            x = res.x if res.status == STAGNATED else np.zeros(n, dtype=wt)
            a *= growth
            restarts += 1
            continue
        return RestartResult(res.x, res.status, used, sum(sum(t.inner_h) for t in attempts),
                             sum(sum(t.inner_s) for t in attempts), a, restarts, attempts)
