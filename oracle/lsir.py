"""Algorithm 2, the refinement loop: augmented-system refinement with split-preconditioned
flexible GMRES (oracle, test use only).

Augmented system (Section 1):  [I A; A^T 0] [r; x] = [b; 0].
Split preconditioner (Section 1):  M_L^-1 = diag(I, R^-T),  M_R^-1 = diag(I, R^-1).

One refinement step i (Algorithm 2):
    residuals:        f = b - r - A x,   g = -A^T r             (precision u_r)
    preconditioned:   h = R^-T g                                (u_r)
    correction:       FGMRES on M_L^-1 Atilde M_R^-1 y = [f; h]; the correction is
             [dr; dx] = Z_k y_k with Z_k = M_R^-1 V_k, so dx = R^-1 dz
    update:           [r; x] += [dr; dx]                        (u)

FGMRES: one cycle, zero initial guess, modified Gram-Schmidt Arnoldi, Givens
rotations; it stops when the preconditioned relative residual estimate
|g_{k+1}| / ||s|| drops to the tolerance (Section 5: "the same values as for
LSQR") or after ``maxit`` (50) iterations.

Residual precision u_r: "f64" (binary64) or "ld" (x87 extended, unit
roundoff 2^-64).  Section 5 pairs u = double with u_r = quad (u_r = u^2);
with u_r = binary64 the residual r cannot be refined below roughly
u_64 ||b|| / ||r||, so the all-binary64 method uses the extended option.

Refinement stops (Section 5 measures against the true solution; that is
offered through ``x_ref``/``r_ref``) when both relative errors are at most
``tol``; without a reference, when both relative corrections
||dx||/||x|| and ||dr||/||r|| are at most ``tol``.  At most ``maxit`` (30)
refinement steps.
"""

import numpy as np

from .qr import solve_upper, solve_upper_t


def fgmres_split(A: np.ndarray, R: np.ndarray, f: np.ndarray, h: np.ndarray,
                 tol: float, maxit: int):
    """Flexible GMRES on M_L^-1 Atilde M_R^-1 with right-hand side s = [f; h].

    Returns (dr, dx, its, relres_estimate).
    """
    m, n = A.shape
    s = np.concatenate([f, h])
    beta = np.linalg.norm(s)
    if beta == 0.0:
        return np.zeros(m), np.zeros(n), 0, 0.0
    V = [s / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    k = 0
    relres = 1.0
    for j in range(maxit):
        vj = V[j]
        z = np.concatenate([vj[:m], solve_upper(R, vj[m:])])          # M_R^-1 v_j
        Z.append(z)
        w_r = z[:m] + A @ z[m:]                                        # Atilde z
        w_x = A.T @ z[:m]
        w = np.concatenate([w_r, solve_upper_t(R, w_x)])              # M_L^-1 (.)
        for i in range(j + 1):                                         # MGS
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0.0:
            V.append(w / H[j + 1, j])
        # apply previous rotations, then a new one eliminating H[j+1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        d = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
        H[j, j] = d
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        relres = abs(g[j + 1]) / beta
        if relres <= tol or len(V) <= j + 1:
            break
    y = solve_upper(H[:k, :k], g[:k])
    corr = np.array(Z[:k]).T @ y
    return corr[:m], corr[m:], k, relres


def lsir(At: np.ndarray, b: np.ndarray, R: np.ndarray, x0: np.ndarray, r0=None,
         tol: float = 1e-12, maxit: int = 30, fgmres_tol: float = 1e-12,
         fgmres_maxit: int = 50, x_ref=None, r_ref=None, u_r: str = "f64"):
    """Refinement loop of Algorithm 2 in binary64 (residuals in ``u_r``).

    Returns (x, r, info).
    """
    A = np.asarray(At, dtype=np.float64).T
    wide = np.longdouble if u_r == "ld" else np.float64
    Aw = np.asarray(At, dtype=wide).T
    bw = np.asarray(b, dtype=wide)
    Rw = np.asarray(R, dtype=wide)
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x if r0 is None else np.array(r0, dtype=np.float64, copy=True)   # the starting residual
    info = dict(its=0, fgmres_its=[], converged=False, relres=[])

    def errs():
        ex = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
        er = np.linalg.norm(r - r_ref) / np.linalg.norm(r_ref)
        return ex, er

    if x_ref is not None and max(errs()) <= tol:
        info["converged"] = True
        return x, r, info
    for i in range(maxit):
        xw, rw = x.astype(wide), r.astype(wide)
        f = (bw - rw - Aw @ xw)                             # residuals in u_r
        g = -(Aw.T @ rw)
        h = solve_upper_t(Rw, g).astype(np.float64)         # h = R^-T g in u_r
        f = f.astype(np.float64)
        dr, dx, k, rr = fgmres_split(A, R, f, h, fgmres_tol, fgmres_maxit)   # the FGMRES correction
        info["fgmres_its"].append(k)
        info["relres"].append(rr)
        r = r + dr                                          # the update
        x = x + dx
        info["its"] = i + 1
        if x_ref is not None:
            done = max(errs()) <= tol
        else:
            nx, nr = np.linalg.norm(x), np.linalg.norm(r)
            done = (np.linalg.norm(dx) <= tol * nx) and (np.linalg.norm(dr) <= tol * nr)
        if done:
            info["converged"] = True
            break
    return x, r, info
