"""The whole method in binary64, and the Section 4.1 condition numbers
(oracle, test use only).

``solve`` runs Algorithm 1 (sketch, Householder R) and Algorithm 2 (LSQR
from the sketch-and-solve point, then augmented-system refinement).

``kappa_aug_closed_form`` is the Section 4.1 expression for the condition
number of the preconditioned augmented matrix [alpha I, B; B^T, 0] with
B = A R^-1, in terms of the extreme singular values of B.

``kappa_est`` and ``terms_for`` choose how many narrow-format parts the
sketch of [A b] needs for Section 4's condition kappa(A) u_s < 1
(``solve(max_terms=...)`` applies them).
"""

import numpy as np

from . import lsir as _lsir
from . import lsqr as _lsqr
from . import qr as _qr
from . import sketch as _sketch


# Unit roundoff of the narrow sketch formats (t fraction bits: 2^-(t+1)).
UNIT_ROUNDOFF = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11, "e4m3": 2.0 ** -4}


def kappa_est(R):
    """||R||_F ||R^-1||_F / sqrt(n) for upper-triangular R (binary64).

    Since kappa_2(R) <= ||R||_F ||R^-1||_F <= n kappa_2(R), the value is within
    a factor sqrt(n) of kappa_2(R) either way; kappa_2(R) = kappa_2(Omega A) is
    kappa(A) up to the embedding's distortion (Section 2).
    """
    R = np.triu(np.asarray(R, dtype=np.float64))
    n = R.shape[0]
    Rinv = np.linalg.inv(R)
    return float(np.linalg.norm(R, "fro") * np.linalg.norm(Rinv, "fro") / np.sqrt(n))


def terms_for(kappa, fmt, terms, max_terms):
    """Parts for the next sketch: Section 4 asks for kappa(A) u_s < 1, and a
    representation of [A b] by `terms` rounded parts in a format of unit
    roundoff u has u_s = u^terms; one more part while the condition fails
    (at most max_terms; binary64 sketches have a single part)."""
    u = UNIT_ROUNDOFF.get(fmt)
    if u is None or terms >= max_terms:
        return terms
    return terms if kappa * u ** terms <= 1.0 else terms + 1


def solve(At, b, s, seed, prob=0, fmt="f64", terms=1, colscale=False,
          lsqr_tol=1e-14, lsqr_maxit=None, lsir_tol=1e-15, lsir_maxit=30,
          fgmres_tol=1e-12, fgmres_maxit=50, x_ref=None, r_ref=None, u_r="ld", timings=None,
          max_terms=0):
    """Sketch -> R -> x^s -> LSQR -> LSIR.  Returns (x, r, info).  With
    max_terms > terms the sketch and R are formed again with one more part
    while terms_for(kappa_est(R), ...) asks for it."""
    import time
    n = At.shape[0]
    t_sk = t_qr = 0.0
    while True:
        t0 = time.perf_counter()
        Y, e = _sketch.sketch(At, b, s, seed, prob, fmt, terms, colscale)
        t1 = time.perf_counter()
        Raug = _qr.householder_r(Y)
        t_sk += t1 - t0
        t_qr += time.perf_counter() - t1
        if max_terms <= terms:
            break
        kest = kappa_est(Raug[:n, :n])
        nxt = terms_for(kest, fmt, terms, max_terms)
        if nxt == terms:
            break
        terms = nxt
    t1 = time.perf_counter()
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
        timings.update(sketch=t_sk, qr=t_qr + (t2 - t1), lsqr=t3 - t2, lsir=t4 - t3)
    return x, r, dict(R=R, Raug=Raug, xs=xs, x0=x0, lsqr=linfo, lsir=rinfo, col_exp=e, terms=terms)


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
