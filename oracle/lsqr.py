"""Algorithm 2, the LSQR solve: LSQR right-preconditioned with R (oracle, test use only).

LSQR is Paige and Saunders' Golub-Kahan bidiagonalisation method (ACM TOMS
8(1), 1982).  It is applied to B = A R^-1 (right preconditioning) in
residual form: starting from the sketch-and-solve point x^s,

    min_y || r_s - B y ||,   r_s = b - A x^s,   x = x^s + R^-1 y.

Stopping (Section 5: "at most 2n iterations or until the tolerance reaches
1e-6 / 1e-12"; the tolerance is read as the two Paige-Saunders
tests with atol = btol = tol):

    ||r_k|| <= tol ||b||        or        ||B^T r_k|| / (||B||_F,est ||r_k||) <= tol

with the recurrence estimates ||r_k|| = phibar_{k+1},
||B^T r_k|| = phibar_{k+1} alpha_{k+1} |c_k| and
||B||_F,est^2 = sum (alpha_i^2 + beta_{i+1}^2).
"""

import numpy as np

from .qr import solve_upper, solve_upper_t


def lsqr_precond(At: np.ndarray, b: np.ndarray, R: np.ndarray, x0: np.ndarray,
                 tol: float, maxit: int, record=False):
    """Preconditioned LSQR from x0.  Returns (x, info dict)."""
    A = np.asarray(At, dtype=np.float64).T
    b = np.asarray(b, dtype=np.float64)
    x0 = np.asarray(x0, dtype=np.float64)
    n = A.shape[1]
    normb = np.linalg.norm(b)

    u = b - A @ x0
    beta = np.linalg.norm(u)
    y = np.zeros(n)
    info = dict(its=0, normr=beta, normar=0.0, normB=0.0, stop="zero-residual", history=[])
    if beta == 0.0:
        return x0.copy(), info
    u /= beta
    v = solve_upper_t(R, A.T @ u)
    alpha = np.linalg.norm(v)
    if alpha == 0.0:
        info["stop"] = "zero-gradient"
        return x0.copy(), info
    v /= alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    normB2 = 0.0
    its = 0
    stop = "maxit"
    for its in range(1, maxit + 1):
        # bidiagonalisation step
        u = A @ solve_upper(R, v) - alpha * u
        beta = np.linalg.norm(u)
        normB2 += alpha * alpha + beta * beta
        if beta > 0.0:
            u /= beta
            v = solve_upper_t(R, A.T @ u) - beta * v
            alpha = np.linalg.norm(v)
            if alpha > 0.0:
                v /= alpha
        # plane rotation eliminating beta
        rho = np.hypot(rhobar, beta)
        c, sn = rhobar / rho, beta / rho
        theta = sn * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = sn * phibar
        y = y + (phi / rho) * w
        w = v - (theta / rho) * w
        normr = phibar
        normar = phibar * alpha * abs(c)
        normB = np.sqrt(normB2)
        if record:
            info["history"].append((its, normr, normar, normB))
        if normr <= tol * normb:
            stop = "test1"
            break
        if normar <= tol * normB * normr:
            stop = "test2"
            break
        if beta == 0.0 or alpha == 0.0:
            stop = "breakdown"
            break
    x = x0 + solve_upper(R, y)
    info.update(its=its, normr=phibar, normar=phibar * alpha * abs(c), normB=np.sqrt(normB2),
                stop=stop, y=y)
    return x, info
