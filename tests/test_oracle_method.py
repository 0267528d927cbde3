"""Pins of the oracle's method steps against mathematics, libraries and the
paper's printed numbers (CPU only)."""

import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg as spla

from conftest import read_golden
from lsdata import make_paper_problem, make_problem
from oracle import formats, lsir, lsqr, philox, qr, refsolve, sketch, solve


# ---------------------------------------------------------------- sketch
def test_sketch_matches_exact_rational_triple_loop():
    P = make_problem(13, 3, 10.0, seed=11, store="f64")
    s = 5
    Y, e = sketch.sketch(P.At, P.b, s, seed=77, prob=2, fmt="f64")
    S = philox.gaussian_block(77, 2, 0, s, 0, 13)
    M = np.column_stack([P.A(), P.b])
    for k in range(s):
        for j in range(4):
            exact = sum(Fraction(float(S[k, i])) * Fraction(float(M[i, j])) for i in range(13))
            assert abs(float(exact) / math.sqrt(s) - Y[k, j]) <= 1e-15 * (1 + abs(Y[k, j]))


@pytest.mark.parametrize("fmt,terms", [("bf16", 1), ("bf16", 2), ("f16", 1), ("e4m3", 2)])
def test_quantised_sketch_is_product_of_quantised_operands(fmt, terms):
    P = make_problem(301, 4, 100.0, seed=5, store="f32")
    s = 9
    colscale = fmt in ("f16", "e4m3")
    Y, e = sketch.sketch(P.At, P.b, s, seed=3, fmt=fmt, terms=terms, colscale=colscale, chunk=64)
    # S from its definition: the 16-bit uniform of entry (k, i) from the Philox
    # block (i // 8, k, 0, 2), through Phi^-1 (mpmath's erfinv), rounded
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    S = np.empty((s, 301))
    for k in range(s):
        for q in range(0, 301, 8):
            w = philox.philox4x32_10(q // 8, k, 0, 2, 3, 0)
            for t in range(min(8, 301 - q)):
                U = (int(w[t // 2]) >> (16 * (t % 2))) & 0xFFFF
                S[k, q + t] = float(mpmath.sqrt(2) * mpmath.erfinv(mpmath.mpf(2 * U + 1) / 65536 - 1))
    Sq = formats.round_to(S, fmt)
    M = np.column_stack([P.A(), P.b.astype(np.float64)])
    Ms = M * 2.0 ** e
    Mq = sum(formats.split_terms(Ms, fmt, terms))
    ref = (Sq @ Mq) / math.sqrt(s) / 2.0 ** e
    assert np.allclose(Y, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    # every scaled, quantised entry is a finite value of the format
    assert np.all(np.isfinite(Mq)) and np.abs(Mq).max() <= formats.FORMATS[fmt][2]
    # and the quantised sketch approximates the one with unrounded operands
    # (the same Gaussian values, [A b] exact) to the format's accuracy
    Y64 = (S @ M) / math.sqrt(s)
    u = formats.UNIT_ROUNDOFF[fmt]
    rel = np.linalg.norm(Y - Y64) / np.linalg.norm(Y64)
    assert rel < 8 * u


def test_sketch_rows_equal_full_sketch_rows():
    P = make_problem(1000, 6, 10.0, seed=2, store="f32")
    Y, _ = sketch.sketch(P.At, P.b, 20, seed=9, fmt="bf16", terms=2, chunk=128)
    rows = [0, 7, 19]
    Yr = sketch.sketch_rows(P.At, P.b, 20, 9, rows, fmt="bf16", terms=2, chunk=333)
    assert np.allclose(Yr, Y[rows], rtol=1e-12, atol=1e-12 * np.abs(Y).max())


def test_sketch_is_a_subspace_embedding():
    # sigma(Omega Q_A) lies near [1 - sqrt(n/s), 1 + sqrt(n/s)] (Marchenko-Pastur);
    # a wrong 1/sqrt(s) scale or a dependent stream would move it.
    P = make_problem(4000, 20, 1.0, seed=8, store="f64")
    Q, _ = np.linalg.qr(P.A())
    Y, _ = sketch.sketch(np.ascontiguousarray(Q.T), np.zeros(4000), 320, seed=4)
    sv = np.linalg.svd(Y[:, :20], compute_uv=False)
    lo, hi = 1 - math.sqrt(20 / 320), 1 + math.sqrt(20 / 320)
    assert lo - 0.08 < sv[-1] and sv[0] < hi + 0.08
    assert abs(np.mean(sv ** 2) - 1.0) < 0.05


# ---------------------------------------------------------------- QR / triangular solves
def _sign_normalise(R):
    return R * np.where(np.diag(R) < 0, -1.0, 1.0)[:, None]


def test_householder_r_matches_lapack_and_gram():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((60, 12)) @ np.diag(np.logspace(0, -4, 12))
    R = qr.householder_r(Y)
    Rl = _sign_normalise(np.linalg.qr(Y, mode="r"))
    assert np.allclose(R, Rl, rtol=1e-10, atol=1e-14)
    assert np.all(np.diag(R) > 0) and np.allclose(R, np.triu(R))
    G = Y.T @ Y
    assert np.linalg.norm(R.T @ R - G) <= 1e-13 * np.linalg.norm(G)


def test_householder_r_special_cases():
    y = np.array([[3.0], [-4.0], [0.0]])
    assert np.allclose(qr.householder_r(y), [[5.0]])
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 5)))
    Rk = np.triu(rng.uniform(1, 2, (5, 5)))
    assert np.allclose(qr.householder_r(Q @ Rk), Rk, atol=1e-13)


def test_triangular_solves_match_lapack():
    rng = np.random.default_rng(4)
    R = np.triu(rng.standard_normal((40, 40))) + 8 * np.eye(40)
    v = rng.standard_normal(40)
    assert np.allclose(qr.solve_upper(R, v), scipy.linalg.solve_triangular(R, v), rtol=1e-12)
    assert np.allclose(qr.solve_upper_t(R, v), scipy.linalg.solve_triangular(R, v, trans="T"),
                       rtol=1e-12)


def test_sketch_and_solve_is_sketched_least_squares():
    P = make_problem(500, 8, 1e3, seed=6, store="f64")
    Y, _ = sketch.sketch(P.At, P.b, 32, seed=1)
    xs = qr.sketch_and_solve(qr.householder_r(Y))
    ref = np.linalg.lstsq(Y[:, :8], Y[:, 8], rcond=None)[0]
    assert np.allclose(xs, ref, rtol=1e-9)


# ---------------------------------------------------------------- LSQR
def _paper_R(P, s, seed):
    Y, _ = sketch.sketch(P.At, P.b, s, seed=seed)
    Raug = qr.householder_r(Y)
    n = P.n
    return Raug[:n, :n], qr.sketch_and_solve(Raug)


def test_lsqr_iterates_match_scipy():
    P = make_problem(800, 30, 1e3, seed=3, store="f64")
    R, xs = _paper_R(P, 120, 5)
    A = P.A()
    B = spla.LinearOperator((800, 30), matvec=lambda y: A @ qr.solve_upper(R, y),
                            rmatvec=lambda u: qr.solve_upper_t(R, A.T @ u), dtype=np.float64)
    r0 = P.b - A @ xs
    for k in (1, 3, 7):
        x, info = lsqr.lsqr_precond(P.At, P.b, R, xs, tol=0.0, maxit=k)
        y_sp = spla.lsqr(B, r0, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
        x_sp = xs + qr.solve_upper(R, y_sp)
        assert info["its"] == k
        assert np.allclose(x, x_sp, rtol=1e-10, atol=1e-12 * np.linalg.norm(x_sp))


def test_lsqr_estimates_match_explicit_norms_and_converge():
    P = make_problem(800, 30, 1e3, seed=4, store="f64")
    R, xs = _paper_R(P, 120, 6)
    A = P.A()
    x, info = lsqr.lsqr_precond(P.At, P.b, R, xs, tol=1e-10, maxit=200, record=True)
    r = P.b - A @ x
    assert abs(np.linalg.norm(r) - info["normr"]) <= 1e-8 * np.linalg.norm(r)
    B = A @ np.linalg.inv(R)
    assert abs(np.linalg.norm(B.T @ r) - info["normar"]) <= 1e-6 * np.linalg.norm(B) * np.linalg.norm(r)
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    ex, er = refsolve.forward_errors(x, r, xr, rr)
    assert ex < 1e-7 and er < 1e-7


# ---------------------------------------------------------------- FGMRES
def test_fgmres_step_k_minimises_over_krylov_space():
    rng = np.random.default_rng(7)
    m, n = 40, 6
    A = rng.standard_normal((m, n))
    R = np.triu(rng.standard_normal((n, n))) + 4 * np.eye(n)
    f, h = rng.standard_normal(m), rng.standard_normal(n)
    Ri = np.linalg.inv(R)
    Mop = np.block([[np.eye(m), A @ Ri], [Ri.T @ A.T, np.zeros((n, n))]])
    s = np.concatenate([f, h])
    for k in (1, 4, 9):
        dr, dx, its, rel = lsir.fgmres_split(A, R, f, h, tol=0.0, maxit=k)
        K = np.column_stack([np.linalg.matrix_power(Mop, i) @ s for i in range(k)])
        c = np.linalg.lstsq(Mop @ K, s, rcond=None)[0]
        y = K @ c
        ours = np.concatenate([dr, R @ dx])        # back to the preconditioned unknowns
        assert its == k
        assert np.allclose(ours, y, rtol=1e-8, atol=1e-9 * np.linalg.norm(y))
        assert abs(rel - np.linalg.norm(s - Mop @ y) / np.linalg.norm(s)) < 1e-9


def test_fgmres_full_dimension_solves_augmented_system():
    rng = np.random.default_rng(8)
    m, n = 12, 4
    A = rng.standard_normal((m, n))
    R = np.triu(rng.standard_normal((n, n))) + 3 * np.eye(n)
    f, g = rng.standard_normal(m), rng.standard_normal(n)
    h = qr.solve_upper_t(R, g)
    dr, dx, its, rel = lsir.fgmres_split(A, R, f, h, tol=1e-15, maxit=m + n)
    At = np.block([[np.eye(m), A], [A.T, np.zeros((n, n))]])
    ref = np.linalg.solve(At, np.concatenate([f, g]))
    assert np.allclose(np.concatenate([dr, dx]), ref, rtol=1e-9, atol=1e-11)


# ---------------------------------------------------------------- reference solver
def test_ref_solve_matches_mpmath_normal_equations():
    P = make_problem(40, 5, 1e4, seed=9, store="f32")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    mpmath.mp.dps = 60
    A = mpmath.matrix([[mpmath.mpf(float(v)) for v in row] for row in P.A()])
    b = mpmath.matrix([mpmath.mpf(float(v)) for v in P.b])
    x = mpmath.lu_solve(A.T * A, A.T * b)
    r = b - A * x
    xm = np.array([float(v) for v in x])
    rm = np.array([float(v) for v in r])
    assert np.linalg.norm(xr - xm) <= 1e-15 * np.linalg.norm(xm)
    assert np.linalg.norm(rr - rm) <= 1e-14 * np.linalg.norm(rm)


def _mpmath_ls(P):
    mpmath.mp.dps = 60
    A = mpmath.matrix([[mpmath.mpf(float(v)) for v in row] for row in P.A()])
    b = mpmath.matrix([mpmath.mpf(float(v)) for v in P.b])
    x = mpmath.lu_solve(A.T * A, A.T * b)
    r = b - A * x
    return np.array([float(v) for v in x]), np.array([float(v) for v in r])


@pytest.mark.parametrize("m,n", [(40, 6), (200, 12)])
def test_ref_solve_matches_mpmath_at_kappa_1e10(m, n):
    # binary64 data with kappa(A) = 1e10 (the m = 5e5, n = 2000 workload's
    # conditioning): the double-double reference equals the 60-digit normal
    # equations solution to binary64 resolution; x87 residuals stall far off
    # (their limiting accuracy, u_ld kappa^2 ||r|| / (||A|| ||x||), is near 1e-4),
    # so the check tells the two apart
    P = make_problem(m, n, 1e10, seed=9, store="f64")
    xm, rm = _mpmath_ls(P)
    xr, rr, info = refsolve.ref_solve(P.At, P.b)
    assert np.linalg.norm(xr - xm) <= 4e-16 * np.linalg.norm(xm)
    assert np.linalg.norm(rr - rm) <= 4e-16 * np.linalg.norm(rm)
    xl, _, _ = refsolve.ref_solve(P.At, P.b, residual="ld")
    assert np.linalg.norm(xl - xm) > 1e-8 * np.linalg.norm(xm)


def test_dd_residual_matches_exact_rationals():
    # f = b - r - A x and g = -A^T r with x, r given as double-double pairs,
    # against exact rational arithmetic: error <= 2^-100 times the sum of the
    # magnitudes of the terms (a double-double's accuracy is about 2^-104)
    rng = np.random.default_rng(21)
    m, n = 9, 4
    A = rng.standard_normal((m, n)) * np.exp(rng.uniform(-8, 8, (m, n)))
    b = rng.standard_normal(m)
    xh = rng.standard_normal(n)
    xl = xh * rng.uniform(-1, 1, n) * 2.0 ** -54
    rh = rng.standard_normal(m) * 1e-3
    rl = rh * rng.uniform(-1, 1, m) * 2.0 ** -54
    At64 = np.ascontiguousarray(A.T)
    fh, fl, gh, gl = refsolve.dd_aug_residual(At64, b, xh, xl, rh, rl)
    F = Fraction
    for i in range(m):
        terms = [F(b[i]), -F(rh[i]), -F(rl[i])] + [-F(A[i, j]) * (F(xh[j]) + F(xl[j])) for j in range(n)]
        exact = sum(terms)
        mag = sum(abs(t) for t in terms)
        assert abs(F(fh[i]) + F(fl[i]) - exact) <= mag * F(2) ** -100
        assert fh[i] == fh[i] + fl[i]                       # normalised pair
    for j in range(n):
        terms = [-F(A[i, j]) * (F(rh[i]) + F(rl[i])) for i in range(m)]
        exact = sum(terms)
        mag = sum(abs(t) for t in terms)
        assert abs(F(gh[j]) + F(gl[j]) - exact) <= mag * F(2) ** -100


def test_ref_solve_recovers_construction_for_exact_storage():
    P = make_problem(3000, 40, 1e2, seed=10, store="f64")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    # f64 storage perturbs the construction only at the 1e-16 * kappa level
    assert np.linalg.norm(xr - P.x_con) <= 1e-12 * np.linalg.norm(P.x_con)
    assert np.linalg.norm(rr - P.r_con) <= 1e-10 * np.linalg.norm(P.r_con)
    assert np.linalg.norm(P.A().T @ rr) <= 1e-13 * np.linalg.norm(P.A()) * np.linalg.norm(rr) * 10


# ---------------------------------------------------------------- Section 4.1 closed form
def test_kappa_closed_form_matches_dense_svd():
    rng = np.random.default_rng(11)
    for alpha in (1.0, 0.3):
        B = rng.standard_normal((30, 6)) @ np.diag([3, 2, 1, 0.5, 0.2, 0.05])
        sv = np.linalg.svd(B, compute_uv=False)
        M = np.block([[alpha * np.eye(30), B], [B.T, np.zeros((6, 6))]])
        direct = np.linalg.cond(M)
        assert abs(solve.kappa_aug_closed_form(sv[0], sv[-1], alpha) / direct - 1) < 1e-10


def test_kappa_aug_of_A_matches_printed_values():
    for row in read_golden("paper_preconditioner_quality.txt"):
        if row[0] == "kappa_aug_A":
            k, printed = float(row[1]), float(row[2])
            val = solve.kappa_aug_closed_form(1.0, 1.0 / k)
            assert abs(val / printed - 1) < 0.005, (k, val, printed)


# ---------------------------------------------------------------- the paper's experiment
def _golden_dict(name):
    return {r[0]: float(r[1]) for r in read_golden(name) if len(r) == 2}


@pytest.mark.slow
def test_preconditioner_quality_matches_paper_statistics():
    gold = _golden_dict("paper_preconditioner_quality.txt")
    vals = []
    for seed in range(6):
        P = make_paper_problem(1000, 100, 1e2, seed)
        R, _ = _paper_R(P, 400, seed + 100)
        nB, nBp, kB = solve.preconditioned_norms(P.At, R)
        vals.append((nB, nBp, kB, solve.kappa_aug_closed_form(nB, 1 / nBp)))
    mean = np.mean(vals, axis=0)
    # seed-to-seed spread (20 seeds): 0.05, 0.014, 0.08, 0.19
    assert abs(mean[0] - gold["norm_AR_inv"]) < 0.15
    assert abs(mean[1] - gold["norm_AR_inv_pinv"]) < 0.05
    assert abs(mean[2] - gold["kappa_AR_inv"]) < 0.25
    assert abs(mean[3] - gold["kappa_precond_augmented"]) < 0.6
    # and Section 2: ||A R^-1|| <= 1/sqrt(1-eps), ||(A R^-1)^+|| <= sqrt(1+eps) with
    # kappa(A R^-1) = kappa(Omega Q_A) independent of kappa(A)
    P2 = make_paper_problem(1000, 100, 1e6, 0)
    R2, _ = _paper_R(P2, 400, 100)
    assert abs(solve.preconditioned_norms(P2.At, R2)[2] / vals[0][2] - 1) < 1e-6


@pytest.mark.slow
def test_lsqr_and_lsir_iteration_counts_match_paper():
    gold = _golden_dict("paper_iteration_counts.txt")
    for seed in (1, 2):
        P = make_paper_problem(1000, 100, 1e2, seed)
        R, xs = _paper_R(P, 400, seed + 100)
        xr, rr, _ = refsolve.ref_solve(P.At, P.b)
        x0, li = lsqr.lsqr_precond(P.At, P.b, R, xs, 1e-6, 200)
        assert abs(li["its"] - gold["lsqr_its"]) <= 2
        ex, er = refsolve.forward_errors(x0, P.b - P.A() @ x0, xr, rr)
        assert gold["lsqr_err_x"] / 5 < ex < gold["lsqr_err_x"] * 5
        assert gold["lsqr_err_r"] / 5 < er < gold["lsqr_err_r"] * 5
        x, r, ri = lsir.lsir(P.At, P.b, R, x0, None, tol=4 * 2.0 ** -24, maxit=30,
                             fgmres_tol=1e-6, fgmres_maxit=50, x_ref=xr, r_ref=rr)
        assert ri["its"] == gold["lsir_its"]
        assert abs(ri["fgmres_its"][0] - gold["fgmres_its"]) <= 5


def test_full_fp64_method_reaches_1e13_on_small_workload():
    P = make_problem(2000, 50, 1e2, seed=2410063190, store="f64")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    x, r, info = solve.solve(P.At, P.b, 200, seed=2410063190)
    ex, er = refsolve.forward_errors(x, r, xr, rr)
    assert ex <= 1e-13 and er <= 1e-13
    # A^T r ~ 0 (normal equations) and kappa(A R^-1) <= 3 for s = 4n
    A = P.A()
    assert np.linalg.norm(A.T @ r) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(r)
    assert solve.preconditioned_norms(P.At, info["R"])[2] <= 3.0
