"""Benchmark: sketch-preconditioned mixed-precision least squares on one MI355X.

One step = one whole solve (narrow-format sketch of [A b] on MFMA, Householder
R, preconditioned LSQR, FGMRES refinement) of a synthetic problem already
resident in HBM.  The headline workload is m = 1e6, n = 1000, s = 4000,
kappa(A) = 1e6, binary32 data, e4m3 sketch with power-of-two column scaling
(three parts), binary64 QR, binary32 LSQR and refinement with binary64
residuals.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--terms T]
                    [--no-cpu-baseline] [--no-fp64] [--no-sparse] [--no-secondary]
"""

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LS solves/s and sketch TFLOP/s at fwd err <=6e-6; mixed vs FP64 speedup"
TARGET_ERR = 6e-6
HBM_PEAK_GBS = 8000.0
# dense MFMA peaks of MI355X by operand format (TFLOP/s)
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f16": 2500.0, "e4m3": 5000.0, "f64": 78.6}
# sketch parts per workload: three e4m3 parts reach the accuracy the e4m3
# MFMA's dot products allow; two bf16 parts bring the m = 1e5 workload to
# kappa u_s < 1
DEFAULT_TERMS = {"fp8_m1M_n1000": 3, "bf16_m100k_n500": 2, "fp64_small": 1, "fp16_m500k_n2000": 1}
SECONDARY = "bf16_m100k_n500"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fp8_m1M_n1000")
    ap.add_argument("--terms", type=int, default=0, help="sketch parts (0: the workload's default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-sparse", action="store_true", help="skip the sparse sign embedding solve")
    ap.add_argument("--no-secondary", action="store_true", help=f"skip the {SECONDARY} figures")
    ap.add_argument("--counter-pass", action="store_true",
                    help="for a rocprofv3 --pmc run: a 256 MiB device copy (calibration), then one solve")
    return ap.parse_args()


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2410_06319_amd", "csrc", f) for f in ("iter.hip", "common.h")]


def traffic_file(workload):
    tag = {"fp8_m1M_n1000": "m1M_n1000", "bf16_m100k_n500": "m100k_n500"}.get(workload, workload)
    return os.path.join(ROOT, "profiles", f"fgmres_pass_{tag}_traffic.md")


TRAFFIC_FILE = traffic_file("bf16_m100k_n500")


def kernel_source_hash():
    """Hash of the code of the FGMRES pass's sources, with comments and blank
    lines removed (a comment edit does not change the kernels)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def recorded_traffic(path=None):
    """HBM bytes per launch of the FGMRES pass from a committed counter
    summary, or None when it is absent or was taken on other kernel sources."""
    try:
        with open(path or TRAFFIC_FILE) as fh:
            kv = dict(line.split("=", 1) for line in fh.read().split() if "=" in line)
        if kv.get("source_sha256_16") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # threadpoolctl missing: report the visible CPUs
        return os.cpu_count() or 1


def cpu_baseline(wl, P, seed, terms):
    """The oracle as it stands, timed on the host on a bounded sample of the
    workload: its first m' rows (m' = m / f, f chosen so the sample stays near
    10-30 s of CPU work).  The sketch, LSQR and refinement stages read A once
    per product, so their times are scaled by f; the QR of the s x (n+1)
    sketch does not depend on m and is reported as measured."""
    from oracle import solve as osolve
    m = wl["m"]
    f = max(1, m // 50000)
    mp = m // f
    At = P.At[:, :mp].copy()
    b = P.b[:mp].copy()
    t = {}
    t0 = time.perf_counter()
    osolve.solve(At, b, wl["s"], seed, fmt=wl["u_s"], terms=terms, colscale=wl["u_s"] in ("f16", "e4m3"),
                 lsqr_tol=1e-6, lsir_tol=TARGET_ERR, fgmres_tol=1e-6, u_r="f64", timings=t)
    wall = time.perf_counter() - t0
    scaled = {k: v * (1 if k == "qr" else f) for k, v in t.items()}
    total = sum(scaled.values())
    return {"value": 1.0 / total, "unit": "solves/s", "cores": int(blas_threads()), "kind": "oracle",
            "sample": (f"the oracle's whole solve (float64 numpy: sketch, Householder R, LSQR, FGMRES refinement) "
                       f"of the workload's first {mp} of {m} rows (n={wl['n']}, s={wl['s']}); {wall:.1f} s of CPU "
                       f"work; sketch, LSQR and refinement times scaled x{f} (linear in m), QR as measured"),
            "stage_s_sample": {k: round(v, 3) for k, v in t.items()},
            "stage_s_scaled": {k: round(v, 3) for k, v in scaled.items()}}


def kernel_table(L, At, b, s, seed, terms, pr, lsir_tol, lsqr_tol):
    """Per-kernel device times (HIP events that each launch stamps with its own
    start and end, on the library's stream) of one solve in the timed
    configuration; the library files only the launches before convergence."""
    Sp = L.Solver(At, b, s=s, seed=seed, terms=terms, pr=pr, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol, profile=1)
    Sp()
    pst = Sp.stats.as_dict()
    del Sp
    kms, kn, kw = pst["kernel_ms"], pst["kernel_launches"], pst["kernel_work"]
    kernels = {}
    for c in kms:
        if kn[c]:
            avg = kms[c] / kn[c]
            if c == "sketch_mfma":
                ach = kw[c] / (kms[c] * 1e-3) / 1e12
                kernels[c] = dict(launches=kn[c], avg_us=1e3 * avg, achieved=ach, unit="TFLOP/s",
                                  flops_per_launch=kw[c] / kn[c])
            else:
                ach = kw[c] / (kms[c] * 1e-3) / 1e9
                kernels[c] = dict(launches=kn[c], avg_us=1e3 * avg, achieved=ach, unit="GB/s",
                                  bytes_per_launch=kw[c] / kn[c])
    return kernels, kms


def timed(S, steps, warmup):
    import torch
    for _ in range(warmup):
        S()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        S()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_workload(L, name, terms, steps, warmup, want_fp64, want_sparse, want_adaptive):
    """Measure one workload; returns (dict of figures, the problem, the reference solution)."""
    import torch
    from lsdata import WORKLOADS, data_seed, make_problem
    from oracle import refsolve

    wl = dict(WORKLOADS[name])
    seed = data_seed(wl["index"])
    m, n, s, kappa = wl["m"], wl["n"], wl["s"], wl["kappa"]
    log(f"[bench] generating {name}: m={m} n={n} s={s} kappa={kappa:g}")
    P = make_problem(m, n, kappa, seed, store=wl["store"])
    At = torch.from_numpy(P.At).cuda()
    b = torch.from_numpy(P.b).cuda()
    mixed = wl["u"] == "f32"
    u_r = wl["u_r"] if mixed else "f64x2"
    pr = L.precs(u_s=wl["u_s"], u_qr=wl["u_qr"], u=wl["u"], u_r=u_r, u_A=wl.get("u_A"))
    lsir_tol = TARGET_ERR if mixed else 1e-15
    lsqr_tol = 1e-6 if mixed else 1e-14
    S = L.Solver(At, b, s=s, seed=seed, terms=terms, pr=pr, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol)
    log(f"[bench] {name}: {warmup} warmup, {steps} timed solves")
    dt = timed(S, steps, warmup)
    st = S.stats.as_dict()
    x = S.x.cpu().numpy()
    r = S.r.cpu().numpy()
    del S
    log(f"[bench] {name}: timed region {dt:.3f} s; reference solution")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b, maxit=4)
    ex, er = refsolve.forward_errors(x, r, xr, rr)
    ok = ex <= TARGET_ERR and er <= TARGET_ERR
    ms = 1e3 * dt / steps
    kernels, kms = kernel_table(L, At, b, s, seed, terms, pr, lsir_tol, lsqr_tol)
    dom = max((c for c in kernels), key=lambda c: kms[c])
    kd = kernels[dom]
    if kd["unit"] == "TFLOP/s":
        peak = MFMA_PEAK_TFLOPS[wl["u_s"]]
        roof = dict(kernel=dom, bound="mfma", achieved=kd["achieved"], peak=peak, unit="TFLOP/s",
                    frac=kd["achieved"] / peak, traffic=None)
    else:
        roof = dict(kernel=dom, bound="hbm", achieved=kd["achieved"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=kd["achieved"] / HBM_PEAK_GBS,
                    traffic=recorded_traffic(traffic_file(name)) if dom == "fgmres_pass" else None)
    sk = kernels.get("sketch_mfma", {})
    sketch_tflops = sk.get("achieved")
    out = {
        "value": (steps / dt) if ok else 0.0, "ms_per_step": ms, "fwd_err_x": ex, "fwd_err_r": er,
        "meets_target": ok,
        "config": {"workload": name, "m": m, "n": n, "s": s, "kappa": kappa, "store": wl["store"],
                   "u_s": wl["u_s"], "terms": terms, "u_qr": wl["u_qr"], "u": wl["u"], "u_r": u_r,
                   "u_A": wl.get("u_A", wl["u"])},
        "sketch_tflops": sketch_tflops,
        "sketch_mfma_frac": (sketch_tflops / MFMA_PEAK_TFLOPS[wl["u_s"]]) if sketch_tflops else None,
        "sketch_mfma_issued_frac": (terms * sketch_tflops / MFMA_PEAK_TFLOPS[wl["u_s"]]) if sketch_tflops else None,
        "iterations": {"lsqr": st["lsqr_its"], "lsir": st["lsir_its"], "fgmres": st["fgmres_its_total"]},
        "stage_ms": {k: round(st[k], 4) for k in ("ms_sketch", "ms_qr", "ms_lsqr", "ms_lsir")},
        "kernels": kernels,
        "roofline": roof,
    }
    if want_fp64 and mixed:
        # the all-binary64 GPU path on the same problem: binary64 MFMA sketch,
        # binary64 QR, LSQR and FGMRES, double-double residuals; one warm-up
        # solve, then the median of three
        pr64 = L.precs(u_s="f64", u_qr="f64", u="f64", u_r="f64x2")
        S64 = L.Solver(At, b, s=s, seed=seed, terms=1, pr=pr64, lsir_tol=TARGET_ERR, lsqr_tol=1e-6)
        log(f"[bench] {name}: all-binary64 GPU path, 1 warmup + 3 solves")
        S64()
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            S64()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
        t64 = statistics.median(times)
        e64 = refsolve.forward_errors(S64.x.cpu().numpy(), S64.r.cpu().numpy(), xr, rr)
        s64 = S64.stats.as_dict()
        out["fp64_path"] = {"ms": 1e3 * t64, "ms_each": [round(1e3 * v, 3) for v in times], "fwd_err_x": e64[0],
                            "fwd_err_r": e64[1],
                            "iterations": {"lsqr": s64["lsqr_its"], "lsir": s64["lsir_its"],
                                           "fgmres": s64["fgmres_its_total"]},
                            "stage_ms": {k: round(s64[k], 3) for k in ("ms_sketch", "ms_qr", "ms_lsqr", "ms_lsir")}}
        out["speedup_vs_fp64"] = (t64 / (dt / steps)) if ok else None
        del S64
    if want_adaptive and mixed:
        # the same solve with the inner FGMRES tolerance relaxed after the first
        # refinement step (ls_iter_opts_t.inner_adapt = 1)
        Sa = L.Solver(At, b, s=s, seed=seed, terms=terms, pr=pr, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol, inner_adapt=1)
        ta = timed(Sa, steps, 1) / steps
        ea = refsolve.forward_errors(Sa.x.cpu().numpy(), Sa.r.cpu().numpy(), xr, rr)
        sa = Sa.stats.as_dict()
        out["adaptive_inner"] = {"ms": 1e3 * ta, "solves_per_s": 1.0 / ta, "fwd_err_x": ea[0], "fwd_err_r": ea[1],
                                 "meets_target": ea[0] <= TARGET_ERR and ea[1] <= TARGET_ERR,
                                 "iterations": {"lsqr": sa["lsqr_its"], "lsir": sa["lsir_its"],
                                                "fgmres": sa["fgmres_its_total"]}}
        del Sa
    if want_sparse and mixed:
        # the same problem with the sparse sign embedding (Section 2, zeta = 8)
        # in place of the Gaussian sketch: binary64 gather, same QR/LSQR/FGMRES
        prs = L.precs(u_s="f64", u_qr=wl["u_qr"], u=wl["u"], u_r=u_r)
        Ss = L.Solver(At, b, s=s, seed=seed, pr=prs, zeta=8, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol)
        log(f"[bench] {name}: sparse sign embedding, 5 solves")
        ts = timed(Ss, 5, 1) / 5
        es = refsolve.forward_errors(Ss.x.cpu().numpy(), Ss.r.cpu().numpy(), xr, rr)
        ss = Ss.stats.as_dict()
        Sq = L.Solver(At, b, s=s, seed=seed, pr=prs, zeta=8, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol, profile=1)
        Sq()
        qs = Sq.stats.as_dict()
        g_ms, g_n, g_w = (qs[k]["sparse_sketch"] for k in ("kernel_ms", "kernel_launches", "kernel_work"))
        out["sparse_sign"] = {
            "zeta": 8, "ms": 1e3 * ts, "solves_per_s": 1.0 / ts, "fwd_err_x": es[0], "fwd_err_r": es[1],
            "stage_ms": {k: round(ss[k], 4) for k in ("ms_sketch", "ms_qr", "ms_lsqr", "ms_lsir")},
            "gather": {"avg_us": 1e3 * g_ms / max(g_n, 1), "achieved": g_w / max(g_ms * 1e-3, 1e-30) / 1e9,
                       "unit": "GB/s", "bytes_per_launch": g_w / max(g_n, 1)},
        }
        del Ss, Sq
    del At, b
    torch.cuda.empty_cache()
    return out, P, seed


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (sharding the problem "
                                   "over several GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    from lsdata import WORKLOADS, data_seed, make_problem
    import paper_2410_06319_amd as L

    name = args.workload
    wl = dict(WORKLOADS[name])
    if "m" not in wl:
        raise SystemExit("the batched workload has no bench line (tests/test_gpu_full_size.py covers it)")
    terms = args.terms or DEFAULT_TERMS.get(name, 1)
    if args.counter_pass:
        # calibration copy of known size, then one solve with the launch
        # configuration of the timed solves
        seed = data_seed(wl["index"])
        P = make_problem(wl["m"], wl["n"], wl["kappa"], seed, store=wl["store"])
        At, b = torch.from_numpy(P.At).cuda(), torch.from_numpy(P.b).cuda()
        xa = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        ya = torch.empty_like(xa)
        for _ in range(3):
            ya.copy_(xa)
        torch.cuda.synchronize()
        pr = L.precs(u_s=wl["u_s"], u_qr=wl["u_qr"], u=wl["u"], u_r=wl["u_r"], u_A=wl.get("u_A"))
        Sc = L.Solver(At, b, s=wl["s"], seed=seed, terms=terms, pr=pr, lsir_tol=TARGET_ERR, lsqr_tol=1e-6,
                      check_every=1)
        Sc()
        torch.cuda.synchronize()
        print(json.dumps({"counter_pass": True, "workload": name, "copy_bytes": 4 * (64 << 20),
                          "source_sha256_16": kernel_source_hash()}), flush=True)
        return
    res, P, seed = run_workload(L, name, terms, args.steps, args.warmup, not args.no_fp64, not args.no_sparse,
                                name == SECONDARY)
    mixed = wl["u"] == "f32"
    out = {
        "metric": METRIC, "value": res.pop("value"), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{wl['u_s']}+f32+f64" if mixed else "f64", "data": "synthetic",
        "config": res.pop("config"),
    }
    out.update(res)
    if not args.no_secondary and name != SECONDARY:
        # the m = 1e5, n = 500 bf16 workload, reported beside the headline
        sec, _, _ = run_workload(L, SECONDARY, DEFAULT_TERMS[SECONDARY], 20, 3, not args.no_fp64, False, True)
        out["secondary"] = sec
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(wl, P, seed, terms)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
