"""The paper's own experiment on the GPU path (Section 5 setup: m = 1000,
n = 100, s = 4n = 400, A with geometric singular values and ||A|| = 1, b
uniform on (0,1) normalised, A and b stored in single precision).

* Tables 1 and 3 at kappa(A) = 1e2 with single-precision working arithmetic:
  LSQR iteration count and forward errors, then one refinement step and its
  FGMRES iteration count (printed values in tests/golden/paper_iteration_counts.txt).
  The sketch is bf16 x 3 terms (A represented to about 2^-24, as a
  single-precision sketch of A would be).
* Section 3.4's claim over a kappa sweep: kappa(A R^-1) stays near the
  embedding's own value while kappa(A) u_s is small and grows in proportion
  to kappa(A) u_s beyond it; a multi-term split of A restores it.  The GPU
  value is compared with the oracle's on the same quantised operands.
"""

import math

import numpy as np
import pytest
import torch

from lsdata import make_paper_problem
from oracle import lsqr as olsqr, qr as oqr, refsolve, sketch as osketch, solve as osolve

pytestmark = pytest.mark.gpu

U_S = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11, "e4m3": 2.0 ** -4}


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2410_06319_amd as lib
    lib.load()
    return lib


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def golden(name):
    import os
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if len(line) == 2:
                out[line[0]] = float(line[1])
    return out


def _gpu_R(L, P, s, seed, fmt, terms, u_qr="f64"):
    At, b = torch.from_numpy(P.At).cuda(), torch.from_numpy(P.b).cuda()
    Yt = L.ls_sketch(At, b, s, seed=seed, u_s=fmt, terms=terms)
    Raug = host(L.ls_qr_r(Yt, u_qr=u_qr)).T
    return Raug, At, b


@pytest.mark.parametrize("seed", [1, 2])
def test_tables_1_and_3_replica(L, seed):
    gold = golden("paper_iteration_counts.txt")
    P = make_paper_problem(1000, 100, 1e2, seed, store="f32")
    n = P.n
    Raug, At, b = _gpu_R(L, P, 400, seed + 100, "bf16", 3, u_qr="f32")
    R = Raug[:n, :n]
    xs = np.linalg.solve(R, Raug[:n, n])
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    x = torch.from_numpy(xs.copy()).cuda()
    Rt = torch.from_numpy(np.ascontiguousarray(R.T)).cuda()
    rc, st = L.ls_lsqr_precond(At, b, Rt, x, u="f32", lsqr_tol=1e-6)
    x0 = host(x)
    ex, er = refsolve.forward_errors(x0, P.b.astype(np.float64) - P.A() @ x0, xr, rr)
    print(f"seed {seed}: LSQR its {st['lsqr_its']} err x {ex:.2e} r {er:.2e}", flush=True)
    assert rc == 0 and abs(st["lsqr_its"] - gold["lsqr_its"]) <= 2
    assert gold["lsqr_err_x"] / 5 < ex < gold["lsqr_err_x"] * 5
    assert gold["lsqr_err_r"] / 5 < er < gold["lsqr_err_r"] * 5
    # one refinement step (Table 3: one step reaches 4u with 39 FGMRES iterations)
    r = torch.empty(P.m, dtype=torch.float64, device="cuda")
    pr = L.precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64")
    rc, st2 = L.ls_lsir_gmres(At, b, Rt, x, r, pr=pr, lsir_maxit=1, fgmres_tol=1e-6, fgmres_maxit=50)
    ex1, er1 = refsolve.forward_errors(host(x), host(r), xr, rr)
    print(f"seed {seed}: one LSIR step, FGMRES its {st2['fgmres_its_total']} err x {ex1:.2e} r {er1:.2e}",
          flush=True)
    assert abs(st2["fgmres_its_total"] - gold["fgmres_its"]) <= 5
    # the paper's stopping test: forward errors of x and r at most 4u (u = 2^-24),
    # up to the rounding of x and r to single precision
    assert ex1 <= 8 * 2.0 ** -24 and er1 <= 8 * 2.0 ** -24


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
def test_preconditioner_quality_against_kappa_u_s(L, fmt):
    rows = []
    for kappa in (1e0, 1e2, 1e3, 1e4, 1e5, 1e6):
        P = make_paper_problem(1000, 100, kappa, 1, store="f32")
        Raug, _, _ = _gpu_R(L, P, 400, 101, fmt, 1)
        k_gpu = osolve.preconditioned_norms(P.At, Raug[:100, :100])[2]
        Y, _ = osketch.sketch(P.At, P.b, 400, 101, fmt=fmt, terms=1, colscale=(fmt != "bf16"))
        k_orc = osolve.preconditioned_norms(P.At, oqr.householder_r(Y)[:100, :100])[2]
        rows.append((kappa, k_gpu, k_orc))
        print(f"{fmt} kappa(A) {kappa:.0e} kappa*u_s {kappa * U_S[fmt]:.2g}: kappa(A R^-1) gpu {k_gpu:.3g} "
              f"oracle {k_orc:.3g}", flush=True)
    for kappa, k_gpu, k_orc in rows:
        # same quantised operands: the two R differ by binary32 accumulation in the sketch
        assert abs(k_gpu - k_orc) <= 0.05 * k_orc
        ku = kappa * U_S[fmt]
        if ku <= 4:
            assert k_gpu <= 3.5          # the Gaussian embedding's own value (about 2.8 at s = 4n)
        if ku >= 30:
            assert k_gpu >= 5.0          # degraded in proportion to kappa(A) u_s
    ks = [r[1] for r in rows]
    assert ks[-1] > 10 * ks[0]


def test_multi_term_split_restores_preconditioner(L):
    # bf16 at kappa(A) = 1e6 (kappa u_s = 3900): one term degrades kappa(A R^-1)
    # by orders of magnitude, two terms (A to about 2^-16) bring it back
    P = make_paper_problem(1000, 100, 1e6, 1, store="f32")
    k1 = osolve.preconditioned_norms(P.At, _gpu_R(L, P, 400, 101, "bf16", 1)[0][:100, :100])[2]
    k3 = osolve.preconditioned_norms(P.At, _gpu_R(L, P, 400, 101, "bf16", 3)[0][:100, :100])[2]
    print(f"bf16 kappa(A)=1e6: kappa(A R^-1) one term {k1:.3g}, three terms {k3:.3g}", flush=True)
    assert k1 > 100 and k3 < 3.5


def _sweep_golden():
    t1, t3 = {}, {}
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables_1_3_sweep.txt")) as fh:
        for line in fh:
            f = line.split("#", 1)[0].split()
            if not f:
                continue
            if f[0] == "t1":
                t1[float(f[1])] = dict(its={"f16": int(f[2]), "bf16": int(f[3])},
                                       ex={"f16": float(f[4]), "bf16": float(f[5])},
                                       er={"f16": float(f[6]), "bf16": float(f[7])})
            elif f[0] == "t3":
                conv = lambda v: None if v == "-" else int(v.rstrip("*"))
                t3[float(f[1])] = dict(lsir={"f16": conv(f[2]), "bf16": conv(f[3])},
                                       fgmres={"f16": conv(f[4]), "bf16": conv(f[5])})
    return t1, t3


# Tables 1 and 3 over kappa(A) = 1e0 .. 1e7 (Section 5's setup, u = u_QR =
# single): u_s half is the fp16 sketch (one part, column scaling); u_s single
# is the bf16 sketch with three parts (A to about 2^-24).  GPU and oracle work
# on the same quantised operands; both are compared with the printed trends:
# while kappa(A) u_s < 1 LSQR needs about 16 iterations and one refinement
# step of about 39-45 FGMRES iterations reaches 4u; beyond it (half from
# kappa = 1e4) LSQR needs many more iterations (up to the 2n cap) and the
# refinement many more FGMRES iterations or does not converge.
@pytest.mark.parametrize("fmt,terms", [("f16", 1), ("bf16", 3)])
def test_kappa_sweep_tables_1_and_3(L, fmt, terms):
    t1, t3 = _sweep_golden()
    u_s = U_S[fmt] ** terms
    rows = []
    for kappa in sorted(t1):
        P = make_paper_problem(1000, 100, kappa, 1, store="f32")
        n = P.n
        xr, rr, _ = refsolve.ref_solve(P.At, P.b)
        # GPU: sketch, QR in single precision, x^s, LSQR, refinement
        Raug, At, b = _gpu_R(L, P, 400, 101, fmt, terms, u_qr="f32")
        R = Raug[:n, :n]
        xs = np.linalg.solve(R, Raug[:n, n])
        x = torch.from_numpy(xs.copy()).cuda()
        Rt = torch.from_numpy(np.ascontiguousarray(R.T)).cuda()
        rc1, st1 = L.ls_lsqr_precond(At, b, Rt, x, u="f32", lsqr_tol=1e-6, lsqr_maxit=200)
        x0 = host(x)
        ex1, er1 = refsolve.forward_errors(x0, P.b.astype(np.float64) - P.A() @ x0, xr, rr)
        r = torch.empty(P.m, dtype=torch.float64, device="cuda")
        pr = L.precs(u_s=fmt, u_qr="f32", u="f32", u_r="f64")
        # Section 5's stopping test: forward errors of x and r against the
        # true solution at most 4u (the reference passed as x_ref, r_ref)
        xr_d, rr_d = torch.from_numpy(xr).cuda(), torch.from_numpy(rr).cuda()
        rc3, st3 = L.ls_lsir_gmres(At, b, Rt, x, r, pr=pr, fgmres_tol=1e-6, fgmres_maxit=50, lsir_maxit=30,
                                   lsir_tol=4 * 2.0 ** -24, x_ref=xr_d.data_ptr(), r_ref=rr_d.data_ptr())
        ex3, er3 = refsolve.forward_errors(host(x), host(r), xr, rr)
        if rc3 == 0:   # the library's own forward errors agree with the host's
            assert st3["err_x"] == pytest.approx(ex3, rel=1e-6) and st3["err_r"] == pytest.approx(er3, rel=1e-6)
        # oracle on the same quantised operands
        Y, _ = osketch.sketch(P.At, P.b, 400, 101, fmt=fmt, terms=terms, colscale=(fmt == "f16"))
        Ro = oqr.householder_r(Y)
        xo, info = olsqr.lsqr_precond(P.At, P.b, Ro[:n, :n], oqr.sketch_and_solve(Ro), tol=1e-6, maxit=200)
        exo, ero = refsolve.forward_errors(xo, P.b.astype(np.float64) - P.A() @ xo, xr, rr)
        rows.append((kappa, st1["lsqr_its"], info["its"], ex1, exo, er1, ero, rc3, st3["lsir_its"],
                     st3["fgmres_its_total"], ex3, er3))
        g1, g3 = t1[kappa], t3[kappa]
        print(f"{fmt}x{terms} kappa {kappa:.0e} (kappa u_s {kappa * u_s:.2g}): LSQR its gpu {st1['lsqr_its']} "
              f"oracle {info['its']} printed {g1['its'][fmt]}; err x {ex1:.2e}/{exo:.2e} (printed {g1['ex'][fmt]:.2e}), "
              f"r {er1:.2e}/{ero:.2e} (printed {g1['er'][fmt]:.2e}); LSIR status {rc3} steps {st3['lsir_its']} "
              f"fgmres {st3['fgmres_its_total']} (printed {g3['lsir'][fmt]}/{g3['fgmres'][fmt]}) "
              f"err x {ex3:.2e} r {er3:.2e}", flush=True)
    base_fg = rows[0][9]
    for (kappa, its_g, its_o, ex1, exo, er1, ero, rc3, lsir, fg, ex3, er3) in rows:
        g1, g3 = t1[kappa], t3[kappa]
        ku = kappa * u_s
        # GPU and oracle LSQR on the same operands: the same iteration count
        # up to binary32 rounding while the preconditioner is good (beyond,
        # where LSQR crawls, the count follows the rounding of every step)
        if ku < 30:
            assert abs(its_g - its_o) <= max(3, 0.2 * its_o)
        if ku < 0.1:
            # the printed regime kappa(A) u_s < 1: about 16 iterations, errors
            # within a factor 5 of the printed ones, the refinement reaching 4u
            # in the printed number of steps with about as many FGMRES iterations
            assert abs(its_g - g1["its"][fmt]) <= 3
            if kappa <= 1e3:   # where the printed LSQR errors are near the working precision's level
                assert g1["ex"][fmt] / 5 < ex1 < 5 * g1["ex"][fmt] and g1["er"][fmt] / 5 < er1 < 5 * g1["er"][fmt]
            assert rc3 == 0 and ex3 <= 4 * 2.0 ** -24 and er3 <= 4 * 2.0 ** -24
            if g3["lsir"][fmt] == 1:
                assert lsir == 1 and abs(fg - g3["fgmres"][fmt]) <= 6
        elif ku > 30:
            # far beyond it: LSQR needs more iterations (printed 85 at
            # kappa u_s = 4.9 and the 2n cap beyond; here, with binary32
            # accumulation of the fp16 products, twice the well-conditioned count
            # at kappa u_s = 49 and the cap an order later), and the refinement
            # needs several times the FGMRES iterations or does not converge
            assert its_g >= 2 * rows[0][1] and its_o >= 2 * rows[0][2]
            assert rc3 != 0 or fg >= 3 * base_fg
            if ku > 300:
                assert its_g >= 100 and its_o >= 100 and rc3 != 0
