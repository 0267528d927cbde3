"""Synthetic dense tall least-squares problems min ||b - A x||_2.

Two constructions:

* ``make_problem`` -- A = U diag(sigma) V^T with U (m x n) and V (n x n) the
  Q factors (diag(R) > 0) of seeded Gaussian matrices, sigma geometric from 1
  to 1/kappa, a known x* ~ N(0, I) and a residual r* orthogonal to range(A)
  with ||r*|| = rho * ||A x*||; b = A x* + r*.  A and b are then rounded
  (round to nearest even) to the storage precision.  After that rounding x*
  and r* are no longer the exact solution of the *stored* data; the exact
  one comes from the oracle's reference solver.

* ``make_paper_problem`` -- the numerical-experiment workload of Section 5 of
  the paper: a randsvd-like A (geometric singular values, ||A||_2 = 1, Haar
  factors) and b with entries uniform on (0, 1), normalised to unit norm (the
  large-residual case).

Storage layout: A is column major with leading dimension m, i.e. the numpy
array returned is ``At`` of shape (n, m) with ``At[j, i] = A[i, j]``; this is
the layout the C library takes (``A + j*lda + i``).
"""

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 2410063190


def data_seed(workload_index: int, problem_index: int = 0) -> int:
    """Seed of one problem: base + 1000 * workload + problem index."""
    return BASE_SEED + 1000 * int(workload_index) + int(problem_index)


# The five problem families the library is measured on (sizes, conditioning,
# storage and the precision recipe of each solve).
WORKLOADS = {
    "fp64_small": dict(index=0, m=2000, n=50, s=200, kappa=1e2, store="f64",
                       u_s="f64", u_qr="f64", u="f64", u_r="f64"),
    "bf16_m100k_n500": dict(index=1, m=100_000, n=500, s=2000, kappa=1e4, store="f32",
                            u_s="bf16", u_qr="f32", u="f32", u_r="f64"),
    "fp8_m1M_n1000": dict(index=2, m=1_000_000, n=1000, s=4000, kappa=1e6, store="f32",
                          u_s="e4m3", u_qr="f64", u="f32", u_r="f64", u_A="f64"),
    "batched_256": dict(index=3, nprob=256, m_range=(5000, 200_000), n_range=(32, 256),
                        log10_kappa_range=(1.0, 5.0), store="f32",
                        u_s="bf16", u_qr="f32", u="f32", u_r="f64"),
    "fp16_m500k_n2000": dict(index=4, m=500_000, n=2000, s=8000, kappa=1e10, store="f64",
                             u_s="f16", u_qr="f64", u="f32", u_r="f64"),
}


@dataclass
class Problem:
    """One least-squares problem in the library's storage layout."""

    At: np.ndarray            # (n, m): column-major A, lda = m
    b: np.ndarray             # (m,)
    x_con: np.ndarray         # constructed x* (exact for the unrounded data), float64
    r_con: np.ndarray         # constructed r* (exact for the unrounded data), float64
    sigma: np.ndarray         # singular values used in the construction
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.At.shape[1]

    @property
    def n(self) -> int:
        return self.At.shape[0]

    def A(self) -> np.ndarray:
        """A as an (m, n) float64 array (exact copy of the stored values)."""
        return self.At.T.astype(np.float64)


def _haar_q(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def _store(x: np.ndarray, store: str) -> np.ndarray:
    if store == "f64":
        return np.ascontiguousarray(x, dtype=np.float64)
    if store == "f32":
        return np.ascontiguousarray(x, dtype=np.float32)
    raise ValueError(f"unsupported storage precision {store!r}")


def make_problem(m: int, n: int, kappa: float, seed: int, store: str = "f32",
                 rho: float = 1e-3) -> Problem:
    """A = U diag(sigma) V^T, x* ~ N(0, I), r* orthogonal to range(A)."""
    if not (m >= n >= 1):
        raise ValueError("need m >= n >= 1")
    rng = np.random.default_rng(np.random.PCG64(seed))
    U = _haar_q(rng, m, n)
    V = _haar_q(rng, n, n)
    if n > 1:
        sigma = float(kappa) ** (-np.arange(n) / (n - 1))
    else:
        sigma = np.ones(1)
    # A^T = V diag(sigma) U^T, built directly in the (n, m) layout.
    At = (V * sigma) @ U.T
    x = rng.standard_normal(n)
    w = rng.standard_normal(m)
    r = w - U @ (U.T @ w)
    Ax = At.T @ x
    r *= rho * np.linalg.norm(Ax) / np.linalg.norm(r)
    b = Ax + r
    return Problem(At=_store(At, store), b=_store(b, store), x_con=x, r_con=r,
                   sigma=sigma, seed=seed,
                   meta=dict(kind="usv", m=m, n=n, kappa=kappa, store=store, rho=rho))


def make_paper_problem(m: int, n: int, kappa: float, seed: int, store: str = "f64") -> Problem:
    """Section 5 workload: randsvd-like A (||A|| = 1), b ~ U(0,1) normalised."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    U = _haar_q(rng, m, n)
    V = _haar_q(rng, n, n)
    sigma = float(kappa) ** (-np.arange(n) / (n - 1)) if n > 1 else np.ones(1)
    At = (V * sigma) @ U.T
    b = rng.uniform(0.0, 1.0, m)
    b /= np.linalg.norm(b)
    nan = np.full(n, np.nan)
    return Problem(At=_store(At, store), b=_store(b, store), x_con=nan, r_con=np.full(m, np.nan),
                   sigma=sigma, seed=seed,
                   meta=dict(kind="paper", m=m, n=n, kappa=kappa, store=store))


def make_batch_sizes(nprob: int = 256, seed: int = BASE_SEED + 3,
                     m_range=(5000, 200_000), n_range=(32, 256),
                     log10_kappa_range=(1.0, 5.0)):
    """Sizes of the uneven batch: m, n uniform integers, log10(kappa) uniform."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    ms = rng.integers(m_range[0], m_range[1] + 1, nprob)
    ns = rng.integers(n_range[0], n_range[1] + 1, nprob)
    lk = rng.uniform(log10_kappa_range[0], log10_kappa_range[1], nprob)
    return [dict(m=int(a), n=int(c), s=4 * int(c), kappa=float(10.0 ** k))
            for a, c, k in zip(ms, ns, lk)]
