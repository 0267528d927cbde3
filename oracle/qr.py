"""Algorithm 1, the QR of the sketch: economic Householder QR, R factor only (oracle, test use only).

Householder QR as in Golub and Van Loan (the analysis of Section 3.1 uses
its standard backward error result): for column j the reflector
P = I - beta v v^T maps Y[j:, j] to alpha e_1 with alpha = -sign(y_1) ||y||,
and is applied to the trailing columns.  Q is never formed (Section 4 notes
that only the R factor is needed).  The rows of R are then scaled by the
signs of its diagonal so that diag(R) > 0, which makes R unique for a
full-rank Y.

Also: back substitution with R (x = R^-1 v) and forward substitution with
R^T (x = R^-T v), the two triangular solves Algorithm 2 uses.
"""

import numpy as np


def householder_r(Y: np.ndarray) -> np.ndarray:
    """R factor (ncol x ncol, upper triangular, diag >= 0) of an s x ncol matrix Y."""
    W = np.array(Y, dtype=np.float64, copy=True)
    s, ncol = W.shape
    if s < ncol:
        raise ValueError("need at least as many rows as columns")
    for j in range(ncol):
        x = W[j:, j]
        nx = np.linalg.norm(x)
        if nx == 0.0:
            continue
        alpha = -nx if x[0] >= 0 else nx
        v = x.copy()
        v[0] -= alpha
        vv = v @ v
        if vv == 0.0:
            continue
        beta = 2.0 / vv
        W[j:, j:] -= beta * np.outer(v, v @ W[j:, j:])
        W[j + 1:, j] = 0.0
    R = np.triu(W[:ncol, :])
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return R * sgn[:, None]


def solve_upper(R: np.ndarray, v: np.ndarray) -> np.ndarray:
    """x with R x = v, R upper triangular (back substitution, row by row)."""
    n = R.shape[0]
    x = np.array(v, dtype=np.result_type(R, v, np.float64), copy=True)
    for i in range(n - 1, -1, -1):
        x[i] = (x[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


def solve_upper_t(R: np.ndarray, v: np.ndarray) -> np.ndarray:
    """x with R^T x = v, R upper triangular (forward substitution)."""
    n = R.shape[0]
    x = np.array(v, dtype=np.result_type(R, v, np.float64), copy=True)
    for i in range(n):
        x[i] = (x[i] - R[:i, i] @ x[:i]) / R[i, i]
    return x


def sketch_and_solve(R_aug: np.ndarray) -> np.ndarray:
    """x^s = R^-1 (Q^T Omega b): with Y = [Omega A, Omega b] factored together,
    Q^T Omega b is the first n entries of the last column of R_aug."""
    n = R_aug.shape[0] - 1
    return solve_upper(R_aug[:n, :n], R_aug[:n, n])
