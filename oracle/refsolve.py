"""Exact least-squares solution of the stored data (oracle, test use only).

Section 5 measures forward errors against a "true" solution computed in
64-digit arithmetic.  Here the stored A and b (exact in binary64) are
solved by refinement on the augmented system [I A; A^T 0] [r; x] = [b; 0]
(Bjorck's approach, cited in Section 1) with:

* a binary64 Householder QR A = Q1 R1 (LAPACK through numpy: a library
  primitive used as one step);
* residuals f = b - r - A x and g = -A^T r evaluated in double-double
  arithmetic (``oracle/ddresid.c``: error-free products and sums, unit
  roundoff about 2^-104), or, with ``residual="ld"``, in x87 extended
  precision (numpy longdouble, 2^-64);
* the correction of the exactly-preconditioned system: with
  z = R1^-T g and c = Q1^T f,  dx = R1^-1 (c - z),  dr = f - Q1 (c - z);
* r and x kept and updated as double-double (or extended) numbers.

The limiting accuracy of the refinement is set by the residual precision,
about u_r kappa(A)^2 ||r|| / (||A|| ||x||) for x: with double-double
residuals it stays far below binary64 resolution up to kappa(A) ~ 1e10
(the workload of m = 5e5, n = 2000), where the x87 variant stalls near
1e-3.  The refinement stops once the relative correction is below ``tol``
or has stopped contracting; the result is returned rounded to binary64.
"""

import ctypes
import os

import numpy as np

from .qr import solve_upper, solve_upper_t

LD = np.longdouble
_HERE = os.path.dirname(os.path.abspath(__file__))
_DD_LIB = os.path.join(_HERE, "libddresid.so")
_dd = None


def _ddlib():
    """The double-double residual kernel, compiled on first use if absent."""
    global _dd
    if _dd is None:
        if not os.path.exists(_DD_LIB):
            from . import build_dd
            build_dd.build()
        lib = ctypes.CDLL(_DD_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.ls_oracle_dd_aug_residual.restype = None
        lib.ls_oracle_dd_aug_residual.argtypes = [ctypes.c_int64, ctypes.c_int64, dp, ctypes.c_int64, dp,
                                                  dp, dp, dp, dp, dp, dp, dp, dp]
        lib.ls_oracle_dd_axpy1.restype = None
        lib.ls_oracle_dd_axpy1.argtypes = [ctypes.c_int64, dp, dp, dp]
        _dd = lib
    return _dd


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def dd_aug_residual(At64, b64, xh, xl, rh, rl):
    """(f_hi, f_lo, g_hi, g_lo): f = b - r - A x, g = -A^T r in double-double.

    At64: (n, m) C-contiguous binary64 (= column-major A, lda = m)."""
    n, m = At64.shape
    fh, fl = np.empty(m), np.empty(m)
    gh, gl = np.empty(n), np.empty(n)
    _ddlib().ls_oracle_dd_aug_residual(m, n, _p(At64), m, _p(b64), _p(xh), _p(xl), _p(rh), _p(rl),
                                       _p(fh), _p(fl), _p(gh), _p(gl))
    return fh, fl, gh, gl


def _dd_add(h, l, y):
    _ddlib().ls_oracle_dd_axpy1(h.shape[0], _p(h), _p(l), _p(np.ascontiguousarray(y, dtype=np.float64)))


def _ref_solve_dd(At, b, maxit, tol):
    At64 = np.ascontiguousarray(At, dtype=np.float64)
    b64 = np.ascontiguousarray(b, dtype=np.float64)
    n, m = At64.shape
    Q1, R1 = np.linalg.qr(At64.T, mode="reduced")
    x0 = solve_upper(R1, Q1.T @ b64)
    xh, xl = np.ascontiguousarray(x0), np.zeros(n)
    zero = np.zeros(m)
    fh, fl, _, _ = dd_aug_residual(At64, b64, xh, xl, zero, zero)
    rh, rl = fh.copy(), fl.copy()                     # r0 = b - A x0
    info = dict(its=0, steps=[])
    prev = np.inf
    best = None
    for it in range(maxit):
        fh, _, gh, _ = dd_aug_residual(At64, b64, xh, xl, rh, rl)
        z = solve_upper_t(R1, gh)
        dz = Q1.T @ fh - z
        dx = solve_upper(R1, dz)
        dr = fh - Q1 @ dz
        _dd_add(xh, xl, dx)
        _dd_add(rh, rl, dr)
        step = max(np.linalg.norm(dx) / max(np.linalg.norm(xh), 1e-300),
                   np.linalg.norm(dr) / max(np.linalg.norm(rh), 1e-300))
        info["steps"].append(step)
        info["its"] = it + 1
        if best is None or step < best[0]:
            best = (step, xh.copy(), rh.copy())
        if step <= tol:
            break
        # stagnation at the residual precision's limiting accuracy
        if step < 1e-12 and step > 0.5 * prev:
            break
        prev = step
    return best[1], best[2], info


def _ref_solve_ld(At, b, maxit, tol):
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


def ref_solve(At: np.ndarray, b: np.ndarray, maxit: int = 12, tol: float = 1e-18, residual: str = "dd"):
    """(x*, r*, info) for min ||b - A x||, A given as At = A^T (n x m).

    residual: "dd" (double-double, default) or "ld" (x87 extended)."""
    if residual == "dd":
        return _ref_solve_dd(At, b, maxit, tol)
    if residual == "ld":
        return _ref_solve_ld(At, b, maxit, tol)
    raise ValueError(f"unknown residual precision {residual!r}")


def forward_errors(x, r, x_ref, r_ref):
    """Relative 2-norm forward errors of x and r (Section 5)."""
    ex = np.linalg.norm(np.asarray(x, np.float64) - x_ref) / np.linalg.norm(x_ref)
    er = np.linalg.norm(np.asarray(r, np.float64) - r_ref) / np.linalg.norm(r_ref)
    return float(ex), float(er)
