"""The whole method in binary64, and the Section 4.1 condition numbers
(oracle, test use only).

``solve`` runs Algorithm 1 (sketch, Householder R) and Algorithm 2 (LSQR
from the sketch-and-solve point, then augmented-system refinement).

``kappa_aug_closed_form`` is the Section 4.1 expression for the condition
number of the preconditioned augmented matrix [alpha I, B; B^T, 0] with
B = A R^-1, in terms of the extreme singular values of B.
"""

import numpy as np

from . import lsir as _lsir
from . import lsqr as _lsqr
from . import qr as _qr
from . import sketch as _sketch


def solve(At, b, s, seed, prob=0, fmt="f64", terms=1, colscale=False,
          lsqr_tol=1e-14, lsqr_maxit=None, lsir_tol=1e-15, lsir_maxit=30,
          fgmres_tol=1e-12, fgmres_maxit=50, x_ref=None, r_ref=None, u_r="ld", timings=None):
    """Sketch -> R -> x^s -> LSQR -> LSIR.  Returns (x, r, info)."""
    import time
    n = At.shape[0]
    t0 = time.perf_counter()
    Y, e = _sketch.sketch(At, b, s, seed, prob, fmt, terms, colscale)
    t1 = time.perf_counter()
    Raug = _qr.householder_r(Y)
    # Section 3.2: with column scaling the preconditioner is R S^-1; here the
    # scaling was undone on Y already, so R_aug is the R factor of Omega [A b].
    R = Raug[:n, :n]
    xs = _qr.sketch_and_solve(Raug)
    t2 = time.perf_counter()
    x0, linfo = _lsqr.lsqr_precond(At, b, R, xs, lsqr_tol, lsqr_maxit or 2 * n)
    t3 = time.perf_counter()
    x, r, rinfo = _lsir.lsir(At, b, R, x0, None, lsir_tol, lsir_maxit, fgmres_tol, fgmres_maxit,
                             x_ref, r_ref, u_r)
    t4 = time.perf_counter()
    if timings is not None:
        timings.update(sketch=t1 - t0, qr=t2 - t1, lsqr=t3 - t2, lsir=t4 - t3)
    return x, r, dict(R=R, Raug=Raug, xs=xs, x0=x0, lsqr=linfo, lsir=rinfo, col_exp=e)


def kappa_aug_closed_form(smax: float, smin: float, alpha: float = 1.0) -> float:
    """Section 4.1: kappa([alpha I, B; B^T, 0]) from sigma_max(B), sigma_min(B)."""
    num = alpha + np.sqrt(alpha * alpha + 4.0 * smax * smax)
    den = min(2.0 * alpha, np.sqrt(alpha * alpha + 4.0 * smin * smin) - alpha)
    # Section 4.1 writes min{2, ...} for alpha = 1 (the eigenvalue alpha of the
    # (1,1) block contributes 2 alpha after the common factor 1/2 cancels).
    return float(num / den)


def preconditioned_norms(At, R):
    """||A R^-1||, ||(A R^-1)^+||, kappa(A R^-1) by a dense SVD (checks only)."""
    A = np.asarray(At, dtype=np.float64).T
    B = np.linalg.solve(R.T, A.T).T
    sv = np.linalg.svd(B, compute_uv=False)
    return float(sv[0]), float(1.0 / sv[-1]), float(sv[0] / sv[-1])
