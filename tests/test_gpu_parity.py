"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Every input is seeded and synthetic (lsdata); expected values come from the
oracle only.  Tolerances are stated next to each comparison with the
arithmetic that fixes them.
"""

import math

import numpy as np
import pytest
import torch

from lsdata import make_problem
from oracle import formats, lsir as olsir, lsqr as olsqr, philox as ophilox, qr as oqr, refsolve, sketch as osketch
from sketch_check import sketch_ratio

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2410_06319_amd as lib
    lib.load()
    return lib


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sync_print(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ random stream
def test_philox_bit_exact(L):
    rng = np.random.default_rng(1)
    for _ in range(4):
        c = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        k = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        c[0] = min(c[0], 2 ** 32 - 5000)
        got = host(L.ls_philox(c[0], c[1], c[2], c[3], k[0], k[1], 4096))
        ref = np.stack(ophilox.philox4x32_10(np.arange(c[0], c[0] + 4096, dtype=np.uint64), c[1], c[2], c[3],
                                             k[0], k[1]), axis=1).astype(np.int64)
        assert np.array_equal(got, ref)


def test_omega_f64_matches_oracle(L):
    seed, s, m = 2410063190, 37, 1003          # ragged: m not a multiple of 4
    S = host(L.ls_omega(seed, s, m, fmt="f64", prob_id=5)).T
    ref = ophilox.gaussian_block(seed, 5, 0, s, 0, m)
    # binary64 Box-Muller on both sides; library log/sincospi within a few ulp
    assert np.max(np.abs(S - ref)) <= 1e-13


# narrow formats: table values on both sides, every entry equal (ragged m:
# not a multiple of 8, the entries of one Philox block)
@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
def test_omega_narrow_matches_oracle_bitwise(L, fmt):
    seed, s, m = 78, 64, 4099
    S = host(L.ls_omega(seed, s, m, fmt=fmt, prob_id=3)).T
    ref = osketch.quantised_gaussian_block(seed, 3, 0, s, 0, m, fmt)
    nd = int(np.count_nonzero(S != ref))
    sync_print(f"{fmt} Omega entries differing from the oracle: {nd} of {S.size}")
    assert nd == 0
    # all 2^16 table values occur as specified: a sample large enough to hit
    # most of them, each entry one of the format's quantiles
    q = osketch.format_quantiles(fmt)
    assert np.all(np.isin(S, q))


# ------------------------------------------------------------------ sketch
def _sketch_gpu(L, P, s, seed, u_s, terms):
    At = dev(P.At)
    b = dev(P.b)
    return host(L.ls_sketch(At, b, s, seed=seed, u_s=u_s, terms=terms)).T


@pytest.mark.parametrize("m,n,s", [(2000, 50, 200), (3001, 13, 77)])
def test_sketch_f64_matches_oracle(L, m, n, s):
    P = make_problem(m, n, 1e2, seed=11, store="f64")
    Y = _sketch_gpu(L, P, s, 2410063190, "f64", 1)
    ref, _ = osketch.sketch(P.At, P.b, s, 2410063190)
    # binary64 products summed in a different order: |dY| <= few * m * u64 * (|S||M|)/sqrt(s)
    M = np.abs(np.column_stack([P.A(), P.b]))
    S = np.abs(ophilox.gaussian_block(2410063190, 0, 0, s, 0, m))
    bound = (S @ M) / math.sqrt(s)
    assert np.all(np.abs(Y - ref) <= 4 * 2.0 ** -53 * math.sqrt(m) * bound + 1e-300)


def _rows(s):
    return sorted({0, 1, s // 3, s // 2, s - 2, s - 1})


@pytest.mark.parametrize("terms", [1, 2, 3])
@pytest.mark.parametrize("m,n,s", [(5003, 37, 100), (20000, 300, 1200)])
def test_sketch_bf16_matches_oracle(L, terms, m, n, s):
    P = make_problem(m, n, 1e3, seed=12, store="f32")
    At, b = dev(P.At), dev(P.b)
    # sampled rows, every column, against the oracle's rounding scale (binary32
    # accumulation over the library's K-split)
    mx, Y, ratio = sketch_ratio(L, P, At, b, s, 99, "bf16", terms, _rows(s))
    sync_print(f"bf16 sketch terms={terms}: max err/(3 scale) {mx:.3f}, median {np.median(ratio):.3f}")
    assert mx <= 1.0
    # and every entry against the oracle's whole sketch, relative to |S_q||M_q|
    ref, _ = osketch.sketch(P.At, P.b, s, 99, fmt="bf16", terms=terms)
    Mq, _ = osketch.scaled_operand(P.At, P.b, "bf16", terms, False)
    Sq = np.abs(osketch.quantised_gaussian_block(99, 0, 0, s, 0, m, "bf16"))
    err = np.abs(Y - ref) / ((Sq @ np.abs(Mq)) / math.sqrt(s))
    assert np.median(err) < 1e-6


# four and five parts (the automatic tile width narrows to 256 columns where
# 512 would not fit the parts in LDS or registers)
@pytest.mark.parametrize("fmt,terms,store", [("bf16", 4, "f32"), ("bf16", 5, "f32"), ("f16", 4, "f64"),
                                             ("f16", 5, "f32"), ("e4m3", 4, "f32"), ("e4m3", 5, "f64")])
def test_sketch_four_and_five_parts_match_oracle(L, fmt, terms, store):
    m, n, s = 20011, 300, 1200
    P = make_problem(m, n, 1e3, seed=12, store=store)
    mx, _, ratio = sketch_ratio(L, P, dev(P.At), dev(P.b), s, 99, fmt, terms, _rows(s))
    sync_print(f"{fmt} x{terms} {store}: max err/(3 scale) {mx:.3f}, median {np.median(ratio):.3f}")
    assert mx <= 1.0


def test_sketch_bf16_split_reaches_binary32_accuracy(L):
    # the multi-term representation: the bf16 x 2 sketch is as close to the
    # exact sketch as binary32 data allows (relative ~ 2^-16 vs 2^-8 for one term)
    P = make_problem(8000, 20, 1e2, seed=13, store="f32")
    exact = _quantile_sketch(P, 84, 5)
    Sq = osketch.quantised_gaussian_block(5, 0, 0, 84, 0, 8000, "bf16")
    M = np.column_stack([P.A(), P.b.astype(np.float64)])
    exact_q = Sq @ M / math.sqrt(84)        # exact product with the bf16-rounded Omega
    errs = []
    for terms in (1, 2):
        Y = _sketch_gpu(L, P, 84, 5, "bf16", terms)
        errs.append(np.linalg.norm(Y - exact_q) / np.linalg.norm(exact_q))
    sync_print("bf16 sketch error vs exact operands, terms 1/2:", errs)
    assert errs[0] < 8 * 2.0 ** -8 and errs[1] < 8 * 2.0 ** -16
    assert np.linalg.norm(exact_q - exact) / np.linalg.norm(exact) < 2.0 ** -6


# narrow formats with the Section 3.2 column scaling (automatic for f16 and
# e4m3): binary32 or binary64 storage, several terms, ragged m
@pytest.mark.parametrize("fmt", ["f16", "e4m3"])
@pytest.mark.parametrize("m,n,s,store,terms", [(5003, 37, 100, "f32", 1), (5003, 37, 100, "f32", 2),
                                               (3001, 13, 77, "f64", 3), (20000, 300, 1200, "f32", 1),
                                               (20000, 300, 1200, "f32", 3), (6000, 2000, 2100, "f64", 3)])
def test_sketch_narrow_colscaled_matches_oracle(L, fmt, m, n, s, store, terms):
    P = make_problem(m, n, 1e3, seed=12, store=store)
    cols = None if n <= 300 else [0, 1, 511, 512, 1023, 1024, n - 1]
    mx, Y, ratio = sketch_ratio(L, P, dev(P.At), dev(P.b), s, 99, fmt, terms, _rows(s), cols=cols)
    ref, e = osketch.sketch(P.At, P.b, s, 99, fmt=fmt, terms=terms, colscale=True)
    Mq, _ = osketch.scaled_operand(P.At, P.b, fmt, terms, True)
    Sq = np.abs(osketch.quantised_gaussian_block(99, 0, 0, s, 0, m, fmt))
    bound = (Sq @ np.abs(Mq)) / math.sqrt(s) * np.ldexp(1.0, -e.astype(np.int64))[None, :]
    err = np.abs(Y - ref) / bound
    sync_print(f"{fmt} sketch terms={terms} store={store}: max err/(3 scale) {mx:.3f}, median err/bound "
               f"{np.median(err):.3e}, exponents {e.min()}..{e.max()}")
    assert mx <= 1.0
    assert np.median(err) < 1e-6


# every launch shape the planner can take (and the autotuned table's choice)
# computes the same sketch: only the grouping of the binary32 partial sums moves
@pytest.mark.parametrize("fmt,terms,store", [("bf16", 2, "f32"), ("e4m3", 3, "f32"), ("f64", 1, "f64")])
def test_sketch_every_launch_shape_matches_oracle(L, fmt, terms, store):
    m, n, s = 7003, 150, 600
    P = make_problem(m, n, 1e3, seed=14, store=store)
    At, b = dev(P.At), dev(P.b)
    cs = fmt == "e4m3"
    ref, e = osketch.sketch(P.At, P.b, s, 77, fmt=fmt, terms=terms, colscale=cs)
    if fmt == "f64":
        M = np.abs(np.column_stack([P.A(), P.b]))
        Sa = np.abs(ophilox.gaussian_block(77, 0, 0, s, 0, m))
        bound = (Sa @ M) / math.sqrt(s)
        tol_max, tol_med = 4 * 2.0 ** -53 * math.sqrt(m), 4 * 2.0 ** -53 * math.sqrt(m)
    outs = {}
    k = 1
    while L.sketch_plan_info(fmt, k) is not None:
        if fmt == "f64":
            Y = host(L.ls_sketch(At, b, s, seed=77, u_s=fmt, terms=terms, plan=k)).T
            err = np.abs(Y - ref) / bound
            sync_print(f"{fmt} x{terms} plan {k} {L.sketch_plan_info(fmt, k)}: max err/bound {err.max():.3e}")
            assert err.max() < tol_max and np.median(err) < tol_med, k
        else:
            # the rounding scale follows each plan's own K-split length
            mx, Y, _ = sketch_ratio(L, P, At, b, s, 77, fmt, terms, _rows(s), plan=k)
            sync_print(f"{fmt} x{terms} plan {k} {L.sketch_plan_info(fmt, k)}: max err/(3 scale) {mx:.3f}")
            assert mx <= 1.0, k
        outs[k] = Y
        k += 1
    Y0 = host(L.ls_sketch(At, b, s, seed=77, u_s=fmt, terms=terms)).T
    assert any(np.array_equal(Y0, Y) for Y in outs.values())   # the table names one of them


@pytest.mark.parametrize("fmt,store", [("e4m3", "f32"), ("f16", "f64"), ("bf16", "f32")])
def test_sketch_reports_column_exponents(L, fmt, store):
    # the Section 3.2 exponents the sketch applied, against the oracle's (0 for
    # bf16, which is not scaled by default)
    P = make_problem(3001, 21, 1e3, seed=24, store=store)
    e = torch.full((22,), -999, dtype=torch.int32, device="cuda")
    L.ls_sketch(dev(P.At), dev(P.b), 96, seed=3, u_s=fmt, terms=2, col_exp=e)
    M = np.column_stack([P.A(), P.b.astype(np.float64)])
    want = formats.column_exponents(M, fmt) if fmt != "bf16" else np.zeros(22, dtype=np.int32)
    assert np.array_equal(host(e), want)


def _quantile_sketch(P, s, seed):
    # the sketch with the narrow formats' Gaussian values unrounded and [A b]
    # exact: Z[k, i] = Phi^-1((U + 1/2) / 2^16)
    Z = ophilox.normal_quantiles16()[ophilox.uniform16_block(seed, 0, 0, s, 0, P.m)]
    M = np.column_stack([P.A(), P.b.astype(np.float64)])
    return Z @ M / math.sqrt(s)


def test_sketch_e4m3_needs_column_scaling(L):
    # entries of A are ~ 1/sqrt(m) ~ 1e-2: without scaling most fall into
    # e4m3's subnormal range (2^-9 .. 2^-6) and lose their digits
    P = make_problem(6000, 24, 1e2, seed=21, store="f32")
    exact = _quantile_sketch(P, 96, 3)
    errs = []
    for cs in (1, -1):
        Y = host(L.ls_sketch(dev(P.At), dev(P.b), 96, seed=3, u_s="e4m3", terms=2, col_scale=cs)).T
        errs.append(np.linalg.norm(Y - exact) / np.linalg.norm(exact))
    sync_print("e4m3 x2 sketch error vs exact, scaled / unscaled:", errs)
    assert errs[0] < 0.1 and errs[1] > 3 * errs[0]


# ------------------------------------------------------------------ QR
@pytest.mark.parametrize("u_qr", ["f64", "f32"])
# panel shapes (rows per thread x columns): s = 2048 is the largest with 4
# rows per thread, s = 2049 the smallest with more; s = 3000 takes the
# 8-row, 8-column binary64 panel
@pytest.mark.parametrize("s,ncols,kappa", [(200, 51, 1e2), (2000, 501, 1e2), (1111, 97, 1e4), (2048, 130, 1e3),
                                          (2049, 33, 1e3), (3000, 77, 1e3)])
def test_qr_r_matches_oracle(L, u_qr, s, ncols, kappa):
    P = make_problem(s, ncols, kappa, seed=14, store="f64")
    Y = P.A()                                       # s x ncols with known conditioning
    Rref = oqr.householder_r(Y)
    Rt = L.ls_qr_r(dev(np.ascontiguousarray(Y.T)), u_qr=u_qr)
    R = host(Rt).T
    assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)
    u = 2.0 ** -53 if u_qr == "f64" else U32
    # backward error of Householder QR: ||Y^T Y - R^T R|| <= c n u ||Y||^2
    G = Y.T @ Y
    assert np.linalg.norm(R.T @ R - G) <= 20 * ncols * u * np.linalg.norm(Y, 2) ** 2
    # forward: R_hat R^-1 = I + Gamma with ||Gamma|| <~ c sqrt(n) u kappa (Section 3.1 proof)
    Gam = np.linalg.solve(Rref.T, R.T).T - np.eye(ncols)
    assert np.linalg.norm(Gam, 2) <= 10 * math.sqrt(ncols) * u * kappa


def test_qr_r_wide_matches_oracle(L):
    # 2001 columns (binary64 QR of the sketch of an n = 2000 problem)
    s, ncols = 4100, 2001
    P = make_problem(s, ncols, 1e3, seed=31, store="f64")
    Y = np.ascontiguousarray(P.A())
    R = host(L.ls_qr_r(dev(np.ascontiguousarray(Y.T)), u_qr="f64")).T
    Rref = oqr.householder_r(Y)
    assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)
    u = 2.0 ** -53
    # the bounds of test_qr_r_matches_oracle
    assert np.linalg.norm(R.T @ R - Y.T @ Y) <= 20 * ncols * u * np.linalg.norm(Y, 2) ** 2
    Gam = np.linalg.solve(Rref.T, R.T).T - np.eye(ncols)
    sync_print("wide QR ||R_hat R^-1 - I||:", np.linalg.norm(Gam, 2))
    assert np.linalg.norm(Gam, 2) <= 10 * math.sqrt(ncols) * u * 1e3


def test_qr_r_rank_deficient_is_reported(L):
    Y = np.random.default_rng(3).standard_normal((100, 8))
    Y[:, 5] = 0.0
    with pytest.raises(L.LsError) as e:
        L.ls_qr_r(dev(np.ascontiguousarray(Y.T)), u_qr="f64")
    assert e.value.code == -4


# ------------------------------------------------------------------ LSQR
def _oracle_R(P, s, seed):
    Y, _ = osketch.sketch(P.At, P.b, s, seed)
    Raug = oqr.householder_r(Y)
    return Raug[:P.n, :P.n], oqr.sketch_and_solve(Raug)


# shapes: 4-row binary32 / 2-row binary64 panels with and without a ragged last
# panel, and n covering one to sixteen 64-column loads per lane
# operand 1: B = A R^-1 formed once; operand 2: A's panels with W = R^-1
# applied around each pass (A stored in u)
@pytest.mark.parametrize("m,n", [(3000, 40), (3001, 40), (5003, 500), (1802, 700)])
@pytest.mark.parametrize("store,u,operand", [("f64", "f64", 1), ("f64", "f64", 2), ("f32", "f32", 1),
                                             ("f32", "f32", 2), ("f32", "f64", 1)])
def test_lsqr_iterates_match_oracle(L, store, u, operand, m, n):
    P = make_problem(m, n, 1e3, seed=15, store=store)
    R, xs = _oracle_R(P, max(160, 2 * n), 3)
    for k in (1, 5, 17):
        x = dev(xs.copy())
        rc, st = L.ls_lsqr_precond(dev(P.At), dev(P.b), dev(np.ascontiguousarray(R.T)), x, u=u,
                                   lsqr_tol=1e-300, lsqr_maxit=k, lsqr_operand=operand)
        xr, info = olsqr.lsqr_precond(P.At, P.b, R, xs, tol=0.0, maxit=k)
        got = host(x)
        assert st["lsqr_its"] == k
        # same recurrences: binary64 agrees to rounding; binary32 vectors differ
        # by O(k u32 kappa(A R^-1)) relative
        tol = 1e-11 if u == "f64" else 2e-4
        assert np.linalg.norm(got - xr) <= tol * np.linalg.norm(xr)
        # entry by entry, against the largest entry of the oracle's iterate
        assert np.max(np.abs(got - xr)) <= tol * np.max(np.abs(xr))
        assert abs(st["lsqr_normr"] - info["normr"]) <= tol * 10 * info["normr"]


def _lapack_R(P, s, seed):
    # the preconditioner input of the wide-panel tests: R of the oracle sketch
    # from LAPACK (rows scaled to diag > 0); both sides receive the same R
    Y, _ = osketch.sketch(P.At, P.b, s, seed)
    Raug = np.linalg.qr(Y, mode="r")
    Raug = Raug * np.where(np.diag(Raug) < 0, -1.0, 1.0)[:, None]
    return Raug[:P.n, :P.n], np.linalg.solve(Raug[:P.n, :P.n], Raug[:P.n, P.n])


# panels of 1025..2048 columns (32 loads per lane, no prefetch of the next panel)
@pytest.mark.parametrize("m,n", [(3001, 1500), (4100, 2048)])
@pytest.mark.parametrize("store,u,operand", [("f32", "f32", 1), ("f32", "f32", 2), ("f64", "f64", 1)])
def test_lsqr_wide_panels_match_oracle(L, store, u, operand, m, n):
    P = make_problem(m, n, 1e2, seed=19, store=store)
    R, xs = _lapack_R(P, 2 * n, 3)
    for k in (1, 5):
        x = dev(xs.copy())
        rc, st = L.ls_lsqr_precond(dev(P.At), dev(P.b), dev(np.ascontiguousarray(R.T)), x, u=u,
                                   lsqr_tol=1e-300, lsqr_maxit=k, lsqr_operand=operand)
        xr, info = olsqr.lsqr_precond(P.At, P.b, R, xs, tol=0.0, maxit=k)
        got = host(x)
        assert st["lsqr_its"] == k
        tol = 1e-11 if u == "f64" else 2e-4
        assert np.linalg.norm(got - xr) <= tol * np.linalg.norm(xr)
        # entry by entry, against the largest entry of the oracle's iterate
        assert np.max(np.abs(got - xr)) <= tol * np.max(np.abs(xr))
        assert abs(st["lsqr_normr"] - info["normr"]) <= tol * 10 * info["normr"]


@pytest.mark.parametrize("m,n", [(5003, 1100), (6000, 2000)])
def test_lsir_wide_panels_reach_target(L, m, n):
    P = make_problem(m, n, 1e4, seed=21, store="f32")
    R, xs = _lapack_R(P, 2 * n, 7)
    x0, _ = olsqr.lsqr_precond(P.At, P.b, R, xs, tol=1e-6, maxit=200)
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    x = dev(x0.copy())
    r = torch.empty(P.m, dtype=torch.float64, device="cuda")
    pr = L.precs(u_s="f64", u_qr="f64", u="f32", u_r="f64")
    rc, st = L.ls_lsir_gmres(dev(P.At), dev(P.b), dev(np.ascontiguousarray(R.T)), x, r, pr=pr, lsir_tol=1.5e-6)
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    sync_print(f"wide LSIR n={n}: its {st['lsir_its']} fgmres {st['fgmres_its_total']} err x {ex:.2e} r {er:.2e}")
    assert rc == 0 and ex <= 6e-6 and er <= 6e-6


def test_lsqr_operand_choices_are_checked(L):
    P = make_problem(3000, 40, 1e3, seed=15, store="f64")
    R, xs = _oracle_R(P, 160, 3)
    Rt = dev(np.ascontiguousarray(R.T))
    with pytest.raises(L.LsError) as e:   # A's panels need A stored in u
        L.ls_lsqr_precond(dev(P.At), dev(P.b), Rt, dev(xs.copy()), u="f32", lsqr_operand=2)
    assert e.value.code == -6   # LS_E_UNSUPPORTED
    with pytest.raises(L.LsError) as e:
        L.ls_lsqr_precond(dev(P.At), dev(P.b), Rt, dev(xs.copy()), u="f64", lsqr_operand=3)
    assert e.value.code == -1   # LS_E_ARG
    Q = make_problem(3000, 40, 1e3, seed=15, store="f32")
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")   # u_A = u: no A-path to share
    with pytest.raises(L.LsError) as e:
        L.ls_solve(dev(Q.At), dev(Q.b), s=160, seed=3, pr=pr, lsqr_operand=2)
    assert e.value.code == -6   # LS_E_UNSUPPORTED


# ls_solve on the A-path: LSQR over A's panels (lsqr_operand = 2) and over
# B = A R^-1 (the default) reach the same accuracy with about as many iterations
@pytest.mark.parametrize("m,n,kappa", [(20000, 100, 1e4), (6003, 700, 1e5)])
def test_solve_lsqr_operands_agree(L, m, n, kappa):
    P = make_problem(m, n, kappa, seed=2410064197, store="f32")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64", u_A="f64")
    res = {}
    for op in (1, 2):
        x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=max(4 * n, n + 1), seed=3, terms=3, pr=pr, lsir_tol=6e-6,
                                  lsqr_operand=op)
        ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
        res[op] = (rc, st["lsqr_its"], st["lsqr_normr"], ex, er)
        sync_print(f"m={m} n={n} LSQR operand {op}: status {rc} lsqr {st['lsqr_its']} normr {st['lsqr_normr']:.6e} "
                   f"err x {ex:.2e} r {er:.2e}")
    for rc, _, _, ex, er in res.values():
        assert rc == 0 and ex <= 6e-6 and er <= 6e-6
    assert abs(res[1][1] - res[2][1]) <= 2
    assert abs(res[1][2] - res[2][2]) <= 1e-3 * res[1][2]


def test_lsqr_converges_like_oracle(L):
    P = make_problem(20000, 100, 1e4, seed=16, store="f32")
    R, xs = _oracle_R(P, 400, 4)
    x = dev(xs.copy())
    rc, st = L.ls_lsqr_precond(dev(P.At), dev(P.b), dev(np.ascontiguousarray(R.T)), x, u="f32")
    _, info = olsqr.lsqr_precond(P.At, P.b, R, xs, tol=1e-6, maxit=200)
    sync_print("LSQR its gpu/oracle:", st["lsqr_its"], info["its"])
    assert rc == 0 and abs(st["lsqr_its"] - info["its"]) <= 2


# ------------------------------------------------------------------ refinement
@pytest.mark.parametrize("m,n", [(6000, 60), (6003, 60), (4001, 300)])
@pytest.mark.parametrize("store,u,u_r,target", [("f64", "f64", "f64x2", 1e-13), ("f32", "f32", "f64", 6e-6)])
def test_lsir_reaches_target_from_oracle_start(L, store, u, u_r, target, m, n):
    P = make_problem(m, n, 1e4, seed=17, store=store)
    R, xs = _oracle_R(P, 4 * n, 6)
    x0, _ = olsqr.lsqr_precond(P.At, P.b, R, xs, tol=1e-6, maxit=120)
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    x = dev(x0.copy())
    r = torch.empty(P.m, dtype=torch.float64, device="cuda")
    pr = L.precs(u_s="f64", u_qr="f64", u=u, u_r=u_r)
    rc, st = L.ls_lsir_gmres(dev(P.At), dev(P.b), dev(np.ascontiguousarray(R.T)), x, r, pr=pr,
                             lsir_tol=(target / 4))
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    ox, orr, oinfo = olsir.lsir(P.At, P.b, R, x0, tol=target / 4, fgmres_tol=1e-6 if u == "f32" else 1e-12,
                                u_r="ld" if u_r == "f64x2" else "f64")
    oex, oer = refsolve.forward_errors(ox, orr, xr, rr)
    sync_print(f"LSIR {store}/{u}/{u_r}: gpu its {st['lsir_its']} fgmres {st['fgmres_its_total']} "
               f"err x {ex:.2e} r {er:.2e}; oracle its {oinfo['its']} {oinfo['fgmres_its']} x {oex:.2e} r {oer:.2e}")
    assert rc == 0
    assert ex <= target and er <= target


# ------------------------------------------------------------------ sparse sign embedding
# Same pattern (Philox words, rejection of repeated rows) and the same
# binary64 additions in the same order (sources of a row of Y in increasing
# i): the GPU sketch equals the oracle's bit for bit.  Shapes: ragged m, both
# storage precisions, n + 1 above 1024 (two column sweeps of the gather).
@pytest.mark.parametrize("m,n,s,zeta,store", [(5003, 37, 160, 4, "f32"), (3001, 13, 100, 8, "f64"),
                                              (20000, 300, 1200, 8, "f32"), (4100, 1500, 1600, 2, "f32"),
                                              (2000, 50, 200, 32, "f64")])
def test_sparse_sketch_matches_oracle_bitwise(L, m, n, s, zeta, store):
    P = make_problem(m, n, 1e3, seed=23, store=store)
    Y = host(L.ls_sketch(dev(P.At), dev(P.b), s, seed=77, u_s="f64", zeta=zeta, prob_id=3)).T
    ref = osketch.sparse_sketch(P.At, P.b, s, 77, zeta, prob=3)
    nd = int(np.count_nonzero(Y != ref))
    sync_print(f"sparse sketch m={m} n={n} s={s} zeta={zeta}: entries differing {nd}")
    assert nd == 0


def test_sparse_sketch_rejects_bad_arguments(L):
    P = make_problem(1000, 20, 10.0, seed=1, store="f32")
    At, b = dev(P.At), dev(P.b)
    for kw in (dict(zeta=1), dict(zeta=33), dict(zeta=30)):          # zeta range, 4 zeta <= s
        with pytest.raises(L.LsError):
            L.ls_sketch(At, b, 100, seed=1, u_s="f64", **kw)
    with pytest.raises(L.LsError):
        L.ls_sketch(At, b, 100, seed=1, u_s="bf16", zeta=4)           # binary64 only


@pytest.mark.parametrize("store,u,u_r,target,m,n,s,kappa", [("f32", "f32", "f64", 6e-6, 20000, 100, 400, 1e4),
                                                            ("f64", "f64", "f64x2", 1e-13, 2000, 50, 200, 1e2)])
def test_solve_with_sparse_sketch_reaches_target(L, store, u, u_r, target, m, n, s, kappa):
    P = make_problem(m, n, kappa, seed=2410064193, store=store)
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    pr = L.precs(u_s="f64", u_qr="f32" if u == "f32" else "f64", u=u, u_r=u_r)
    x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=s, seed=9, pr=pr, zeta=8,
                              lsir_tol=target if u == "f32" else 1e-15, lsqr_tol=1e-6 if u == "f32" else 1e-14)
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    sync_print(f"sparse-sketch solve {store}/{u}: lsqr {st['lsqr_its']} lsir {st['lsir_its']} "
               f"fgmres {st['fgmres_its_total']} err x {ex:.2e} r {er:.2e}")
    assert rc == 0 and ex <= target and er <= target


# ------------------------------------------------------------------ whole method
@pytest.mark.parametrize("u_s,terms,u,u_r", [("bf16", 2, "f32", "f64"), ("f16", 2, "f32", "f64"),
                                             ("f64", 1, "f64", "f64x2")])
def test_solve_ignores_prior_workspace_contents(L, u_s, terms, u, u_r):
    # every buffer a step reads is written first: the same solve on a zeroed
    # workspace and on one filled with large or NaN byte patterns agrees bitwise
    P = make_problem(6003, 60, 1e4, seed=2410064192, store="f32")
    pr = L.precs(u_s=u_s, u_qr="f32" if u == "f32" else "f64", u=u, u_r=u_r)
    S = L.Solver(dev(P.At), dev(P.b), s=240, seed=5, terms=terms, pr=pr,
                 lsir_tol=6e-6 if u == "f32" else 1e-15, lsqr_tol=1e-6 if u == "f32" else 1e-14)
    out = []
    for fill in (0x00, 0x7A, 0xFF, 0x00):
        S.ws.fill_(fill)
        rc = S(check=False)
        out.append((rc, host(S.x), host(S.r), S.stats.as_dict()["fgmres_its_total"]))
    sync_print(f"workspace fills {u_s}/{u}: status {[o[0] for o in out]} fgmres {[o[3] for o in out]}")
    for rc, x, r, _ in out:
        assert rc == 0
        assert np.array_equal(x, out[0][1]) and np.array_equal(r, out[0][2])


@pytest.mark.parametrize("fmt,terms,kappa", [("bf16", 2, 1e4), ("e4m3", 3, 1e3)])
def test_adaptive_inner_tolerance_reaches_target_with_fewer_iterations(L, fmt, terms, kappa):
    P = make_problem(20000, 100, kappa, seed=2410064194, store="f32")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    pr = L.precs(u_s=fmt, u_qr="f32", u="f32", u_r="f64")
    res = {}
    for adapt in (0, 1):
        x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=400, seed=7, terms=terms, pr=pr, lsir_tol=6e-6,
                                  inner_adapt=adapt)
        ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
        res[adapt] = (rc, st["lsir_its"], st["fgmres_its_total"], ex, er)
        sync_print(f"{fmt} inner_adapt={adapt}: lsir {st['lsir_its']} fgmres {st['fgmres_its_total']} "
                   f"err x {ex:.2e} r {er:.2e}")
    for rc, _, _, ex, er in res.values():
        assert rc == 0 and ex <= 6e-6 and er <= 6e-6
    assert res[1][2] < res[0][2]


def test_solve_fp64_workload_reaches_1e13(L):
    P = make_problem(2000, 50, 1e2, seed=2410063190, store="f64")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    pr = L.precs(u_s="f64", u_qr="f64", u="f64", u_r="f64x2")
    x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=200, seed=2410063190, pr=pr, lsqr_tol=1e-14,
                              lsir_tol=1e-15)
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    sync_print("fp64 solve:", st, ex, er)
    assert rc == 0 and ex <= 1e-13 and er <= 1e-13


def test_solve_mixed_bf16_reaches_6e6(L):
    P = make_problem(20000, 100, 1e4, seed=2410064190, store="f32")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")
    x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=400, seed=7, terms=2, pr=pr, lsir_tol=6e-6)
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    sync_print("mixed solve:", st, ex, er)
    assert rc == 0 and ex <= 6e-6 and er <= 6e-6


@pytest.mark.parametrize("fmt,terms,kappa", [("f16", 2, 1e4), ("e4m3", 3, 1e3)])
def test_solve_narrow_sketch_reaches_6e6(L, fmt, terms, kappa):
    P = make_problem(20000, 100, kappa, seed=2410064191, store="f32")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    pr = L.precs(u_s=fmt, u_qr="f32", u="f32", u_r="f64")
    x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=400, seed=8, terms=terms, pr=pr, lsir_tol=6e-6)
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    sync_print(f"{fmt} x{terms} solve:", st["lsqr_its"], st["lsir_its"], st["fgmres_its_total"], ex, er)
    assert rc == 0 and ex <= 6e-6 and er <= 6e-6


@pytest.mark.parametrize("kappa,want_terms", [(1e1, 1), (1e4, 2)])
def test_solve_adds_sketch_parts_while_kappa_u_s_exceeds_one(L, kappa, want_terms):
    # bf16 from one part with max_terms = 3: kappa(A) = 1e4 gives kappa_est u_s
    # near 40 with one part and 0.15 with two, so the solve settles on two parts
    # (kappa = 10: one part suffices).  The reported estimate is the oracle's
    # estimate of the R the GPU forms from the sketch with that many parts, and
    # the oracle's rule on the GPU's one-part R asks for the same parts.
    from oracle import solve as osolve
    P = make_problem(20000, 100, kappa, seed=2410064192, store="f32")
    At, b = dev(P.At), dev(P.b)
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")
    x, r, rc, st = L.ls_solve(At, b, s=400, seed=9, terms=1, max_terms=3, pr=pr, lsir_tol=6e-6)
    sync_print(f"kappa {kappa:g}: parts {st['sketch_terms']}, kappa_est {st['kappa_est']:.4g}, "
               f"lsqr {st['lsqr_its']}, fgmres {st['fgmres_its_total']}")
    assert rc == 0 and st["sketch_terms"] == want_terms
    ests = []
    for t in range(1, want_terms + 1):
        Y = L.ls_sketch(At, b, 400, seed=9, u_s="bf16", terms=t)
        R = host(L.ls_qr_r(Y, u_qr="f32")).T[:100, :100]
        ests.append(osolve.kappa_est(R))
    # the same R (deterministic sketch and QR); R^-1 by two routes: binary64
    # rounding amplified by kappa(R) <= 1e4 at most
    assert st["kappa_est"] == pytest.approx(ests[-1], rel=1e-9)
    t = 1
    while osolve.terms_for(ests[t - 1], "bf16", t, 3) != t:
        t += 1
    assert t == want_terms
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    assert ex <= 6e-6 and er <= 6e-6


def test_profile_files_one_record_per_launch_before_convergence(L):
    # profile = 1 with the default queue depth: the launches queued past
    # convergence are not filed, so the counts follow the iteration counts
    P = make_problem(20000, 100, 1e4, seed=2410064193, store="f32")
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")
    x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=400, seed=7, terms=2, pr=pr, lsir_tol=6e-6, profile=1)
    n_l, ms = st["kernel_launches"], st["kernel_ms"]
    sync_print("profile:", n_l, {k: round(v, 3) for k, v in ms.items()})
    assert rc == 0
    assert n_l["sketch_mfma"] == 1
    assert n_l["lsqr_pass"] == st["lsqr_its"] + 2          # the first pass, then iterations 1 .. its + 1
    # a converged cycle of k columns makes k + 1 passes: the stage after the
    # last one finds the convergence of column k - 1
    assert n_l["fgmres_pass"] == st["fgmres_its_total"] + st["lsir_its"]
    assert n_l["cgs_sweep"] == st["fgmres_its_total"] + st["lsir_its"]
    assert n_l["lsir_resid_pass"] == st["lsir_its"]
    for k in ("sketch_mfma", "lsqr_pass", "fgmres_pass", "lsir_resid_pass", "cgs_sweep"):
        assert ms[k] > 0


# degenerate shapes: one column, s = n + 1 (no embedding margin), m = n + 1,
# very few columns with a long ragged m; the oracle converges on each
@pytest.mark.parametrize("m,n,s,kappa", [(200, 1, 4, 1.0), (2000, 20, 21, 10.0), (41, 40, 41, 10.0),
                                         (5000, 3, 12, 1e3)])
def test_solve_degenerate_shapes(L, m, n, s, kappa):
    P = make_problem(m, n, kappa, seed=77, store="f32")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")
    x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=s, seed=5, terms=2, pr=pr, lsir_tol=6e-6)
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    sync_print(f"m={m} n={n} s={s}: lsqr {st['lsqr_its']} lsir {st['lsir_its']} fgmres {st['fgmres_its_total']} "
               f"x {ex:.2e} r {er:.2e}")
    assert rc == 0 and ex <= 6e-6 and er <= 6e-6
    P64 = make_problem(m, n, kappa, seed=77, store="f64")
    xr, rr, _ = refsolve.ref_solve(P64.At, P64.b)
    pr = L.precs(u_s="f64", u_qr="f64", u="f64", u_r="f64x2")
    x, r, rc, st = L.ls_solve(dev(P64.At), dev(P64.b), s=s, seed=5, pr=pr, lsir_tol=1e-15)
    ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
    assert rc == 0 and ex <= 1e-13 and er <= 1e-13


def test_solve_batched_equals_single_solves(L):
    # uneven problems (sizes, conditioning, seeds) over several workers: each
    # result is bitwise the single-problem one and reaches the target
    shapes = [(12000, 60, 1e4), (3001, 17, 1e2), (20000, 120, 1e3), (5000, 33, 1e5), (8003, 90, 1e2),
              (2500, 48, 1e3), (15000, 24, 1e4), (4096, 64, 1e1), (9000, 100, 1e3), (6000, 75, 1e2)]
    probs = [make_problem(m, n, k, seed=2410063190 + 3000 + i, store="f32") for i, (m, n, k) in enumerate(shapes)]
    seeds = [2410063190 + 3000 + i for i in range(len(probs))]
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")
    dev_probs = [(dev(P.At), dev(P.b)) for P in probs]
    xs, rs, rc, stats = L.ls_solve_batched(dev_probs, seeds=seeds, terms=2, pr=pr, nworkers=4, lsir_tol=6e-6)
    assert rc == 0
    for i, (P, (At, b)) in enumerate(zip(probs, dev_probs)):
        # problem i of a batch draws Omega with prob_id = i
        x1, r1, rc1, st1 = L.ls_solve(At, b, s=0, seed=seeds[i], terms=2, pr=pr, prob_id=i, lsir_tol=6e-6)
        assert rc1 == 0 and stats[i]["status"] == 0
        assert torch.equal(xs[i], x1) and torch.equal(rs[i], r1), f"problem {i} differs from its single solve"
        for k in ("lsqr_its", "lsir_its", "fgmres_its_total"):
            assert stats[i][k] == st1[k], (i, k)
        xr, rr, _ = refsolve.ref_solve(P.At, P.b)
        ex, er = refsolve.forward_errors(host(xs[i]), host(rs[i]), xr, rr)
        assert ex <= 6e-6 and er <= 6e-6, (i, ex, er)
    sync_print("batched lsqr its:", [st["lsqr_its"] for st in stats], "fgmres:", [st["fgmres_its_total"] for st in stats])


# HIP graphs: the FGMRES iterations captured in chunks of check_every at a
# call's first refinement step and replayed at the later ones (with eager
# launches, copies and synchronisations between the replays) give bitwise the
# eager result.  Three refinement steps are forced (lsir_tol unreachable), the
# tolerance changes from step to step (inner_adapt), and chunks of 4 leave a
# ragged last one (fgmres_maxit 22); B-path and binary64-product A-path.
@pytest.mark.parametrize("u_A", ["f32", "f64"])
def test_graph_replay_equals_eager_launches(L, u_A):
    P = make_problem(20000, 100, 1e6, seed=2410063190 + 5000, store="f32")
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64", u_A=u_A)
    At, b = dev(P.At), dev(P.b)
    common = dict(s=400, seed=11, terms=1, pr=pr, lsir_tol=1e-300, lsir_maxit=3, fgmres_maxit=22, check_every=4,
                  inner_adapt=1)
    x0, r0, rc0, st0 = L.ls_solve(At, b, graph=0, **common)
    assert st0["lsir_its"] == 3 and st0["fgmres_its_total"] > 22
    for rep in range(2):   # a second call captures its own graphs again
        x1, r1, rc1, st1 = L.ls_solve(At, b, graph=1, **common)
        assert rc1 == rc0 and torch.equal(x1, x0) and torch.equal(r1, r0), f"call {rep} differs from eager"
        for k in ("lsqr_its", "lsir_its", "fgmres_its_total"):
            assert st1[k] == st0[k], (rep, k)
    sync_print(f"graph replay u_A={u_A}: lsir {st0['lsir_its']} fgmres {st0['fgmres_its_total']} (bitwise equal)")


# A batch whose problems fall into several grouped sketch launches (tile widths
# 128, 256 and 512 columns) in e4m3 with column scaling: each result is bitwise
# the problem's single solve (whose sketch is its own launch).
def test_batched_grouped_e4m3_sketches_equal_single_solves(L):
    shapes = [(6000, 40, 1e3), (9001, 200, 1e2), (7000, 300, 1e3), (12000, 70, 1e4), (8000, 260, 1e2)]
    probs = [make_problem(m, n, k, seed=2410063190 + 7000 + i, store="f32") for i, (m, n, k) in enumerate(shapes)]
    seeds = [2410063190 + 7000 + i for i in range(len(probs))]
    pr = L.precs(u_s="e4m3", u_qr="f32", u="f32", u_r="f64")
    dev_probs = [(dev(P.At), dev(P.b)) for P in probs]
    xs, rs, rc, stats = L.ls_solve_batched(dev_probs, seeds=seeds, terms=3, pr=pr, nworkers=2, lsir_tol=6e-6)
    for i, (At, b) in enumerate(dev_probs):
        x1, r1, rc1, st1 = L.ls_solve(At, b, s=0, seed=seeds[i], terms=3, pr=pr, prob_id=i, lsir_tol=6e-6)
        assert stats[i]["status"] == rc1 and stats[i]["sketch_plan"] == st1["sketch_plan"]
        assert torch.equal(xs[i], x1) and torch.equal(rs[i], r1), f"problem {i} differs from its single solve"
    sync_print("grouped e4m3 batch: lsir its", [st["lsir_its"] for st in stats])


def test_batched_with_graphs_equals_single_solves(L):
    shapes = [(12000, 60, 1e4), (3001, 17, 1e2), (20000, 120, 1e5), (5000, 33, 1e5), (8003, 90, 1e2)]
    probs = [make_problem(m, n, k, seed=2410063190 + 6000 + i, store="f32") for i, (m, n, k) in enumerate(shapes)]
    seeds = [2410063190 + 6000 + i for i in range(len(probs))]
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")
    dev_probs = [(dev(P.At), dev(P.b)) for P in probs]
    xs, rs, rc, stats = L.ls_solve_batched(dev_probs, seeds=seeds, terms=2, pr=pr, nworkers=3, lsir_tol=6e-6,
                                           graph=1, check_every=4)
    for i, (At, b) in enumerate(dev_probs):
        x1, r1, rc1, st1 = L.ls_solve(At, b, s=0, seed=seeds[i], terms=2, pr=pr, prob_id=i, lsir_tol=6e-6,
                                      check_every=4)
        assert stats[i]["status"] == rc1
        assert torch.equal(xs[i], x1) and torch.equal(rs[i], r1), f"problem {i} differs from its single solve"
    sync_print("batched with graphs: lsir its", [st["lsir_its"] for st in stats])


def test_batched_lsqr_limit_is_per_problem(L):
    # Section 5's LSQR limit is 2n for each problem: with an unreachable
    # tolerance every problem of a batch stops at its own 2n
    shapes = [(4000, 12), (3001, 40), (5000, 25)]
    probs = [make_problem(m, n, 1e2, seed=2410063190 + 4000 + i, store="f32") for i, (m, n) in enumerate(shapes)]
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")
    dev_probs = [(dev(P.At), dev(P.b)) for P in probs]
    xs, rs, rc, stats = L.ls_solve_batched(dev_probs, seeds=[5, 6, 7], terms=2, pr=pr, lsqr_tol=1e-300,
                                           lsir_maxit=1, nworkers=2)
    assert [st["lsqr_its"] for st in stats] == [2 * n for _, n in shapes]


def test_solve_rejects_bad_arguments(L):
    P = make_problem(100, 10, 10.0, seed=1, store="f32")
    At, b = dev(P.At), dev(P.b)
    with pytest.raises(L.LsError) as e:
        L.ls_solve(At, b, s=5, seed=1, terms=2, pr=L.precs())          # s < n + 1
    assert e.value.code == -1
    with pytest.raises(L.LsError) as e:
        L.ls_solve(At, b, s=40, seed=1, terms=6, pr=L.precs())         # terms out of range
    assert e.value.code == -1
    for terms, max_terms in ((2, 1), (1, 6)):                         # max_terms below terms or above 5
        with pytest.raises(L.LsError) as e:
            L.ls_solve(At, b, s=40, seed=1, terms=terms, max_terms=max_terms, pr=L.precs())
        assert e.value.code == -1
    for plan in (-1, 99):                                             # no such launch shape
        with pytest.raises(L.LsError) as e:
            L.ls_sketch(At, b, 40, seed=1, u_s="bf16", terms=1, plan=plan)
        assert e.value.code == -1


# ------------------------------------------------------------------ binary64 products over A (A-path)
# With u = binary32 and u_A = u_L = u_R = binary64 the FGMRES pass streams a
# panel copy of A (as stored) and applies W = R^-1 on either side, with
# binary64 products: one refinement step of k FGMRES iterations then matches
# the oracle's binary64 step up to the rounding of x and r to binary32.
# Shapes: 4-row panels with a ragged last one, and n from one to sixteen
# 64-column loads per lane (n = 1100: the widest panels, no prefetch; its
# residuals are formed over A as stored, the others' over the panel copy), and
# m = 300001, where the Gram-Schmidt sweeps run over more than 512 row blocks
# and their partial dot products are summed by a launch of their own.
@pytest.mark.parametrize("m,n", [(3001, 40), (4007, 200), (5003, 300), (4001, 700), (6002, 1100), (300001, 24)])
@pytest.mark.parametrize("store", ["f32", "f64"])
def test_refinement_step_with_binary64_products_matches_oracle(L, m, n, store):
    P = make_problem(m, n, 1e4, seed=25, store=store)
    R, xs = _lapack_R(P, 2 * n, 5)
    x0, _ = olsqr.lsqr_precond(P.At, P.b, R, xs, tol=1e-6, maxit=60)
    A = P.A()
    r0 = P.b.astype(np.float64) - A @ x0
    k = 12
    ox, orr, _ = olsir.lsir(P.At, P.b, R, x0, r0=r0, tol=0.0, maxit=1, fgmres_tol=1e-300, fgmres_maxit=k)
    x, r = dev(x0.copy()), dev(r0.copy())
    pr = L.precs(u_s="f64", u_qr="f64", u="f32", u_r="f64", u_A="f64")
    rc, st = L.ls_lsir_gmres(dev(P.At), dev(P.b), dev(np.ascontiguousarray(R.T)), x, r, pr=pr, r_given=True,
                             lsir_maxit=1, lsir_tol=1e-300, fgmres_tol=1e-300, fgmres_maxit=k)
    gx, gr = host(x), host(r)
    assert st["fgmres_its_total"] == k
    # x and r leave the step rounded to binary32 (the working precision)
    ex = np.abs(gx - ox) / (2 * U32 * np.abs(ox) + 1e-9 * np.abs(ox).max())
    er = np.abs(gr - orr) / (2 * U32 * np.abs(orr) + 1e-9 * np.abs(orr).max())
    sync_print(f"A-path step m={m} n={n} {store}: max dev/bound x {ex.max():.3f} r {er.max():.3f}")
    assert ex.max() <= 1.0 and er.max() <= 1.0


@pytest.mark.parametrize("m,n,kappa", [(20000, 100, 1e4), (6003, 700, 1e5), (5003, 1100, 1e4)])
def test_solve_with_binary64_products_reaches_target(L, m, n, kappa):
    P = make_problem(m, n, kappa, seed=2410064196, store="f32")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    res = {}
    for uA in ("f32", "f64"):
        pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64", u_A=uA)
        x, r, rc, st = L.ls_solve(dev(P.At), dev(P.b), s=max(4 * n, n + 1), seed=3, terms=3, pr=pr, lsir_tol=6e-6)
        ex, er = refsolve.forward_errors(host(x), host(r), xr, rr)
        res[uA] = (rc, st["lsir_its"], st["fgmres_its_total"], ex, er)
        sync_print(f"m={m} n={n} kappa={kappa:.0e} u_A={uA}: status {rc}, lsir {st['lsir_its']}, "
                   f"fgmres {st['fgmres_its_total']}, err x {ex:.2e} r {er:.2e}")
    for rc, _, _, ex, er in res.values():
        assert rc == 0 and ex <= 6e-6 and er <= 6e-6
    # binary64 products need no more refinement steps than binary32 ones
    assert res["f64"][1] <= res["f32"][1]
