"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times.

At these sizes the oracle cannot run the whole method, so each test checks
what it can compute one by one or what holds at any size:

* sampled sketch entries Y[k, j] (each costs m multiply-adds in the oracle)
  against the oracle's quantised sketch, relative to |S_q| |M_q| / sqrt(s);
* R^T R = Y^T Y for the R factor the GPU computes from the GPU sketch
  (Householder QR backward stability);
* the whole solve against the reference solution of the stored data
  (forward error <= 6e-6 in x and r).

The 256-problem batch is solved whole; a sample of its problems is checked
against the reference solution.
"""

import math
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from lsdata import WORKLOADS, data_seed, make_batch_sizes, make_problem
from oracle import refsolve, sketch as osketch
from sketch_check import sketch_ratio

pytestmark = pytest.mark.gpu

TARGET = 6e-6
UNIT = {"f32": 2.0 ** -24, "f64": 2.0 ** -53}


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2410_06319_amd as lib
    lib.load()
    return lib


def say(*a):
    print(*a, flush=True)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _sketch_entries(L, At, b, P, s, seed, fmt, terms, rows, cols):
    """Sampled entries of the GPU sketch against the oracle: the GPU sketch and
    err / (2 x the oracle's rounding scale) for the sampled entries."""
    mx, Y, ratio = sketch_ratio(L, P, At, b, s, seed, fmt, terms, rows, cols=cols)
    return Y, ratio


def _qr_backward(L, Y, u_qr):
    Yt = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()
    R = host(L.ls_qr_r(Yt, u_qr=u_qr)).T
    N = Y.shape[1]
    rel = np.linalg.norm(R.T @ R - Y.T @ Y) / np.linalg.norm(Y) ** 2
    return rel, 10.0 * math.sqrt(N) * UNIT[u_qr]


def _run_workload(L, name, terms, rows, cols):
    wl = WORKLOADS[name]
    seed = data_seed(wl["index"])
    t0 = time.time()
    P = make_problem(wl["m"], wl["n"], wl["kappa"], seed, store=wl["store"])
    say(f"{name}: generated {wl['m']} x {wl['n']} in {time.time() - t0:.1f} s")
    At, b = torch.from_numpy(P.At).cuda(), torch.from_numpy(P.b).cuda()
    Y, err = _sketch_entries(L, At, b, P, wl["s"], seed, wl["u_s"], terms, rows, cols)
    say(f"{name}: sketch entries err/(3 scale) max {err.max():.3f} median {np.median(err):.3f}")
    # binary32 accumulation over the library's K-split and the e4m3 MFMA's
    # dot-product window
    assert err.max() <= 1.0
    rel, lim = _qr_backward(L, Y, wl["u_qr"])
    say(f"{name}: |R^T R - Y^T Y| / |Y|^2 = {rel:.3e} (limit {lim:.1e})")
    assert rel <= lim
    pr = L.precs(u_s=wl["u_s"], u_qr=wl["u_qr"], u=wl["u"], u_r=wl["u_r"], u_A=wl.get("u_A"))
    S = L.Solver(At, b, s=wl["s"], seed=seed, terms=terms, pr=pr, lsir_tol=TARGET, lsqr_tol=1e-6)
    rc = S(check=False)
    st = S.stats.as_dict()
    x, r = host(S.x), host(S.r)
    say(f"{name}: status {rc}, lsqr {st['lsqr_its']}, lsir {st['lsir_its']}, fgmres {st['fgmres_its_total']}")
    del S, At, b
    torch.cuda.empty_cache()
    t0 = time.time()
    xr, rr, _ = refsolve.ref_solve(P.At, P.b, maxit=2)
    ex, er = refsolve.forward_errors(x, r, xr, rr)
    say(f"{name}: forward error x {ex:.3e} r {er:.3e} (reference in {time.time() - t0:.1f} s)")
    assert rc == 0 and ex <= TARGET and er <= TARGET


def test_full_size_bf16_workload(L):
    # m=100000 n=500 s=2000 kappa=1e4, binary32 data, bf16 x 2 sketch (the benchmark's solve)
    _run_workload(L, "bf16_m100k_n500", 2, rows=[0, 777, 1999], cols=[0, 1, 255, 256, 498, 499])


def test_full_size_e4m3_workload(L):
    # m=1e6 n=1000 s=4000 kappa=1e6, binary32 data, e4m3 x 3 sketch with column
    # scaling (two terms leave kappa u_s > 1 and the refinement does not converge)
    _run_workload(L, "fp8_m1M_n1000", 3, rows=[0, 2048, 3999], cols=[0, 1, 511, 512, 998, 999])


def test_full_size_sparse_sign_sketch(L):
    # the m=1e5 n=500 s=2000 problem sketched with the sparse sign embedding
    # (zeta = 8): sampled rows of Y equal the oracle's bit for bit, and the
    # solve reaches the target with it
    wl = WORKLOADS["bf16_m100k_n500"]
    seed = data_seed(wl["index"])
    P = make_problem(wl["m"], wl["n"], wl["kappa"], seed, store=wl["store"])
    At, b = torch.from_numpy(P.At).cuda(), torch.from_numpy(P.b).cuda()
    Y = host(L.ls_sketch(At, b, wl["s"], seed=seed, u_s="f64", zeta=8)).T
    rows = [0, 1, 999, 1999]
    ref = osketch.sparse_sketch_rows(P.At, P.b, wl["s"], seed, 8, rows)
    assert np.array_equal(Y[rows], ref)
    pr = L.precs(u_s="f64", u_qr="f32", u="f32", u_r="f64")
    S = L.Solver(At, b, s=wl["s"], seed=seed, pr=pr, zeta=8, lsir_tol=TARGET, lsqr_tol=1e-6)
    rc = S(check=False)
    st = S.stats.as_dict()
    x, r = host(S.x), host(S.r)
    say(f"sparse sign: status {rc}, lsqr {st['lsqr_its']}, lsir {st['lsir_its']}, fgmres {st['fgmres_its_total']}, "
        f"sketch {st['ms_sketch']:.3f} ms")
    del S, At, b
    torch.cuda.empty_cache()
    xr, rr, _ = refsolve.ref_solve(P.At, P.b, maxit=2)
    ex, er = refsolve.forward_errors(x, r, xr, rr)
    say(f"sparse sign: forward error x {ex:.3e} r {er:.3e}")
    assert rc == 0 and ex <= TARGET and er <= TARGET


def test_full_size_batch_of_256(L):
    # 256 problems, m in [5000, 200000], n in [32, 256], s = 4n, kappa in
    # [1e1, 1e5]: solved in one call; every problem converges, sampled ones are
    # checked against the reference solution
    wl = WORKLOADS["batched_256"]
    sizes = make_batch_sizes()
    t0 = time.time()

    def gen(i):
        d = sizes[i]
        return make_problem(d["m"], d["n"], d["kappa"], data_seed(wl["index"], i), store=wl["store"])

    # each problem has its own seed: threads (numpy releases the GIL in its
    # generators and LAPACK) give the same arrays as a serial loop
    probs = [None] * len(sizes)
    with ThreadPoolExecutor(max_workers=8) as ex:
        for i, P in enumerate(ex.map(gen, range(len(sizes)))):
            probs[i] = P
            if (i + 1) % 64 == 0:
                say(f"batch: generated {i + 1} problems ({time.time() - t0:.1f} s)")
    dev_probs = [(torch.from_numpy(P.At).cuda(), torch.from_numpy(P.b).cuda()) for P in probs]
    seeds = [data_seed(wl["index"], i) for i in range(len(probs))]
    pr = L.precs(u_s=wl["u_s"], u_qr=wl["u_qr"], u=wl["u"], u_r=wl["u_r"])
    # bf16 x 3 keeps kappa u_s < 1 up to kappa = 1e5
    xs, rs, rc, stats = L.ls_solve_batched(dev_probs, seeds=seeds, terms=3, pr=pr, lsir_tol=TARGET)
    torch.cuda.synchronize()
    t1 = time.time()
    xs, rs, rc, stats = L.ls_solve_batched(dev_probs, seeds=seeds, terms=3, pr=pr, lsir_tol=TARGET)
    torch.cuda.synchronize()
    dt = time.time() - t1
    bad = [i for i, st in enumerate(stats) if st["status"] != 0]
    say(f"batch: status {rc}, {len(probs) / dt:.1f} problems/s, not converged {bad}")
    assert rc == 0 and not bad
    kap = [d["kappa"] for d in sizes]
    ms = [d["m"] for d in sizes]
    sample = sorted({int(np.argmax(kap)), int(np.argmax(ms)), int(np.argmin(ms)), 0, 100, 200})
    for i in sample:
        P = probs[i]
        xr, rr, _ = refsolve.ref_solve(P.At, P.b, maxit=2)
        ex, er = refsolve.forward_errors(host(xs[i]), host(rs[i]), xr, rr)
        say(f"batch problem {i} (m={P.m} n={P.n} kappa={sizes[i]['kappa']:.2e}): x {ex:.3e} r {er:.3e}")
        assert ex <= TARGET and er <= TARGET


# ------------------------------------------------------------------ kappa = 1e10, binary64 data
@pytest.fixture(scope="module")
def cfg4():
    # m = 5e5, n = 2000, kappa = 1e10, binary64 storage (8 GB), and the exact
    # solution of the stored data (double-double refinement)
    wl = WORKLOADS["fp16_m500k_n2000"]
    seed = data_seed(wl["index"])
    t0 = time.time()
    P = make_problem(wl["m"], wl["n"], wl["kappa"], seed, store=wl["store"])
    say(f"kappa 1e10 workload: generated {wl['m']} x {wl['n']} in {time.time() - t0:.1f} s")
    t0 = time.time()
    xr, rr, info = refsolve.ref_solve(P.At, P.b, maxit=6)
    say(f"kappa 1e10 workload: reference in {time.time() - t0:.1f} s, steps {['%.1e' % v for v in info['steps']]}")
    return wl, seed, P, xr, rr


def _cfg4_solve(L, cfg4, pr, terms, **opts):
    wl, seed, P, xr, rr = cfg4
    At, b = torch.from_numpy(P.At).cuda(), torch.from_numpy(P.b).cuda()
    S = L.Solver(At, b, s=wl["s"], seed=seed, terms=terms, pr=pr, **opts)
    t0 = time.time()
    rc = S(check=False)
    torch.cuda.synchronize()
    dt = time.time() - t0
    st = S.stats.as_dict()
    x, r = host(S.x), host(S.r)
    del S, At, b
    torch.cuda.empty_cache()
    ex, er = refsolve.forward_errors(x, r, xr, rr)
    say(f"  status {rc}, {dt * 1e3:.0f} ms, kappa_est {st['kappa_est']:.3g}, lsqr {st['lsqr_its']}, lsir {st['lsir_its']}, "
        f"fgmres {st['fgmres_its_total']}, err x {ex:.3e} r {er:.3e}, stages "
        f"{[round(st[k], 1) for k in ('ms_sketch', 'ms_qr', 'ms_lsqr', 'ms_lsir')]} ms")
    return rc, st, ex, er, dt


def test_full_size_fp16_workload_as_written(L, cfg4):
    # fp16 sketch (one part, column scaling), binary64 QR, binary32 LSQR and
    # FGMRES products, binary64 residuals.  kappa(A) u = 1e10 2^-24 ~ 600 and
    # kappa(A) u_s ~ 5e6 lie outside the conditions of Section 4 (and of the
    # refinement's limiting accuracy with binary64 residuals); Table 4 prints
    # "-" for u_s half and single at kappa = 1e10 even with u = double.  The
    # library reports LS_NOT_CONVERGED with finite iterates.
    say("kappa 1e10 as written (fp16 x1, u = binary32):")
    pr = L.precs(u_s="f16", u_qr="f64", u="f32", u_r="f64")
    rc, st, ex, er, _ = _cfg4_solve(L, cfg4, pr, 1, lsir_tol=6e-6, lsqr_tol=1e-6)
    assert rc == 1
    assert np.isfinite(ex) and np.isfinite(er)


def test_full_size_fp16_workload_binary64_path(L, cfg4):
    # the all-binary64 path on the same problem (binary64 MFMA sketch, QR,
    # LSQR and FGMRES; double-double residuals): Table 4's u_s = double column
    # converges at kappa = 1e10 (2 steps, 100 FGMRES iterations)
    say("kappa 1e10, all binary64:")
    pr = L.precs(u_s="f64", u_qr="f64", u="f64", u_r="f64x2")
    rc, st, ex, er, dt = _cfg4_solve(L, cfg4, pr, 1, lsir_tol=1e-12, lsqr_tol=1e-12)
    assert rc == 0 and ex <= TARGET and er <= TARGET
