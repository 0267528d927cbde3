"""Exact least-squares solution of the stored data (oracle, test use only).

Section 5 measures forward errors against a "true" solution computed in
64-digit arithmetic.  Here the stored A and b (exact in binary64) are
solved by refinement on the augmented system [I A; A^T 0] [r; x] = [b; 0]
(Bjorck's approach, cited in Section 1) with:

* a binary64 Householder QR A = Q1 R1 (LAPACK through numpy: a library
  primitive used as one step);
* residuals f = b - r - A x and g = -A^T r evaluated in x87 extended
  precision (numpy longdouble, 64-bit significand, unit roundoff 2^-64);
* the correction of the exactly-preconditioned system: with
  z = R1^-T g and c = Q1^T f,  dx = R1^-1 (c - z),  dr = f - Q1 (c - z);
* r and x kept and updated in extended precision.

It converges while kappa(A)^2 * 2^-64 << 1, which covers every problem with
kappa <= 1e6.  The result is returned rounded to binary64.
"""

import numpy as np

from .qr import solve_upper, solve_upper_t

LD = np.longdouble


def ref_solve(At: np.ndarray, b: np.ndarray, maxit: int = 12, tol: float = 1e-18):
    """(x*, r*, info) for min ||b - A x||, A given as At = A^T (n x m)."""
    if np.finfo(LD).nmant < 63:
        raise RuntimeError("extended precision (x87 long double) is not available")
    A64 = np.asarray(At, dtype=np.float64).T
    b64 = np.asarray(b, dtype=np.float64)
    Q1, R1 = np.linalg.qr(A64, mode="reduced")
    Ald = np.asarray(At, dtype=LD).T
    bld = b64.astype(LD)
    c0 = Q1.T @ b64
    x = solve_upper(R1, c0).astype(LD)
    r = bld - Ald @ x
    info = dict(its=0, steps=[])
    for it in range(maxit):
        f = (bld - r - Ald @ x)
        g = -(Ald.T @ r)
        f64 = f.astype(np.float64)
        g64 = g.astype(np.float64)
        z = solve_upper_t(R1, g64)
        c = Q1.T @ f64
        dz = c - z
        dx = solve_upper(R1, dz)
        dr = f64 - Q1 @ dz
        x = x + dx.astype(LD)
        r = r + dr.astype(LD)
        step = max(np.linalg.norm(dx) / max(np.linalg.norm(x.astype(np.float64)), 1e-300),
                   np.linalg.norm(dr) / max(np.linalg.norm(r.astype(np.float64)), 1e-300))
        info["steps"].append(step)
        info["its"] = it + 1
        if step <= tol:
            break
    return x.astype(np.float64), r.astype(np.float64), info


def forward_errors(x, r, x_ref, r_ref):
    """Relative 2-norm forward errors of x and r (Section 5)."""
    ex = np.linalg.norm(np.asarray(x, np.float64) - x_ref) / np.linalg.norm(x_ref)
    er = np.linalg.norm(np.asarray(r, np.float64) - r_ref) / np.linalg.norm(r_ref)
    return float(ex), float(er)
