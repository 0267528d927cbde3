"""Benchmark: sketch-preconditioned mixed-precision least squares on one MI355X.

One step = one whole solve (bf16 sketch of [A b] on MFMA, Householder R,
preconditioned LSQR, FGMRES refinement) of a synthetic problem already
resident in HBM.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline] [--no-fp64] [--no-sparse]
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LS solves/s and sketch TFLOP/s at fwd err <=6e-6; mixed vs FP64 speedup"
TARGET_ERR = 6e-6
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f64": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bf16_m100k_n500")
    ap.add_argument("--terms", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-sparse", action="store_true", help="skip the sparse sign embedding solve")
    ap.add_argument("--counter-pass", action="store_true",
                    help="for a rocprofv3 --pmc run: a 256 MiB device copy (calibration), then one solve")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fgmres_pass_m100k_n500_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2410_06319_amd", "csrc", f) for f in ("iter.hip", "common.h")]


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


def recorded_traffic():
    """HBM bytes per launch of the FGMRES pass from the committed counter
    summary, or None when it is absent or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split("=", 1) for line in fh.read().split() if "=" in line)
        if kv.get("source_sha256_16") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(wl, P, seed, terms):
    """The oracle as it stands, timed on the host on one whole solve of the same problem."""
    from oracle import solve as osolve
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # threadpoolctl missing: report the visible CPUs
        cores = os.cpu_count() or 1
    t = {}
    t0 = time.perf_counter()
    osolve.solve(P.At, P.b, wl["s"], seed, fmt=wl["u_s"], terms=terms, lsqr_tol=1e-6,
                 lsir_tol=TARGET_ERR, fgmres_tol=1e-6, u_r="f64", timings=t)
    wall = time.perf_counter() - t0
    return {"value": 1.0 / wall, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"one whole oracle solve (float64 numpy: sketch, Householder R, LSQR, FGMRES refinement) of "
                       f"the same {wl['m']} x {wl['n']} problem (s={wl['s']}, kappa={wl['kappa']:g}); "
                       f"{wall:.1f} s of CPU work"),
            "stage_s": {k: round(v, 3) for k, v in t.items()}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (sharding the problem "
                                   "over several GPUs is not implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch
    from lsdata import WORKLOADS, data_seed, make_problem
    import paper_2410_06319_amd as L
    from oracle import refsolve

    wl = dict(WORKLOADS[args.workload])
    if "m" not in wl:
        raise SystemExit("the batched workload has no bench line (tests/test_gpu_full_size.py covers it)")
    seed = data_seed(wl["index"])
    m, n, s, kappa = wl["m"], wl["n"], wl["s"], wl["kappa"]
    terms = args.terms if wl["u_s"] == "bf16" else 1
    log(f"[bench] generating {args.workload}: m={m} n={n} s={s} kappa={kappa:g}")
    P = make_problem(m, n, kappa, seed, store=wl["store"])
    At = torch.from_numpy(P.At).cuda()
    b = torch.from_numpy(P.b).cuda()
    mixed = wl["u"] == "f32"
    u_r = wl["u_r"] if mixed else "f64x2"
    pr = L.precs(u_s=wl["u_s"], u_qr=wl["u_qr"], u=wl["u"], u_r=u_r)
    lsir_tol = TARGET_ERR if mixed else 1e-15
    lsqr_tol = 1e-6 if mixed else 1e-14
    if args.counter_pass:
        # calibration copy of known size, then one solve with the launch
        # configuration of the profiled solve below
        xa = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        ya = torch.empty_like(xa)
        for _ in range(3):
            ya.copy_(xa)
        torch.cuda.synchronize()
        Sc = L.Solver(At, b, s=s, seed=seed, terms=terms, pr=pr, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol, check_every=1)
        Sc()
        torch.cuda.synchronize()
        print(json.dumps({"counter_pass": True, "copy_bytes": 4 * (64 << 20), "source_sha256_16": kernel_source_hash()}),
              flush=True)
        return
    S = L.Solver(At, b, s=s, seed=seed, terms=terms, pr=pr, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol)
    for _ in range(args.warmup):
        S()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup}); timing {args.steps} solves")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = S.stats.as_dict()
    x = S.x.cpu().numpy()
    r = S.r.cpu().numpy()
    log(f"[bench] timed region {dt:.3f} s; reference solution")
    xr, rr, _ = refsolve.ref_solve(P.At, P.b)
    ex, er = refsolve.forward_errors(x, r, xr, rr)
    ok = ex <= TARGET_ERR and er <= TARGET_ERR
    ms = 1e3 * dt / args.steps
    value = (args.steps / dt) if ok else 0.0

    # Per-kernel device times (HIP events that each launch stamps with its own
    # start and end, on the library's stream), same problem and launch
    # configuration as the timed solves; the library files only the launches
    # before convergence (those queued beyond it return at once).
    Sp = L.Solver(At, b, s=s, seed=seed, terms=terms, pr=pr, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol, profile=1)
    Sp()
    pst = Sp.stats.as_dict()
    kms, kn, kw = pst["kernel_ms"], pst["kernel_launches"], pst["kernel_work"]
    kernels = {}
    for c in kms:
        if kn[c]:
            avg = kms[c] / kn[c]
            if c == "sketch_mfma":
                ach = kw[c] / (kms[c] * 1e-3) / 1e12
                kernels[c] = dict(launches=kn[c], avg_us=1e3 * avg, achieved=ach, unit="TFLOP/s")
            else:
                ach = kw[c] / (kms[c] * 1e-3) / 1e9
                kernels[c] = dict(launches=kn[c], avg_us=1e3 * avg, achieved=ach, unit="GB/s",
                                  bytes_per_launch=kw[c] / kn[c])
    dom = max((c for c in kernels), key=lambda c: kms[c])
    kd = kernels[dom]
    if kd["unit"] == "TFLOP/s":
        peak = MFMA_PEAK_TFLOPS[wl["u_s"]]
        roof = dict(kernel=dom, bound="mfma", achieved=kd["achieved"], peak=peak, unit="TFLOP/s",
                    frac=kd["achieved"] / peak, traffic=None)
    else:
        roof = dict(kernel=dom, bound="hbm", achieved=kd["achieved"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=kd["achieved"] / HBM_PEAK_GBS,
                    traffic=recorded_traffic() if dom == "fgmres_pass" else None)
    sk = kernels.get("sketch_mfma", {})
    sketch_tflops = sk.get("achieved")

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "s": s, "kappa": kappa, "store": wl["store"],
                   "u_s": wl["u_s"], "terms": terms, "u_qr": wl["u_qr"], "u": wl["u"], "u_r": u_r},
        "fwd_err_x": ex, "fwd_err_r": er, "meets_target": ok,
        "sketch_tflops": sketch_tflops,
        "sketch_mfma_frac": (sketch_tflops / MFMA_PEAK_TFLOPS[wl["u_s"]]) if sketch_tflops else None,
        "iterations": {"lsqr": st["lsqr_its"], "lsir": st["lsir_its"], "fgmres": st["fgmres_its_total"]},
        "stage_ms": {k: round(st[k], 4) for k in ("ms_sketch", "ms_qr", "ms_lsqr", "ms_lsir")},
        "kernels": kernels,
        "roofline": roof,
    }
    if not args.no_fp64 and mixed:
        pr64 = L.precs(u_s="f64", u_qr="f64", u="f64", u_r="f64x2")
        S64 = L.Solver(At, b, s=s, seed=seed, terms=1, pr=pr64, lsir_tol=TARGET_ERR, lsqr_tol=1e-6)
        log("[bench] all-binary64 GPU path, one solve")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        S64()
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        e64 = refsolve.forward_errors(S64.x.cpu().numpy(), S64.r.cpu().numpy(), xr, rr)
        s64 = S64.stats.as_dict()
        out["fp64_path"] = {"ms": 1e3 * t64, "fwd_err_x": e64[0], "fwd_err_r": e64[1],
                            "stage_ms": {k: round(s64[k], 3) for k in ("ms_sketch", "ms_qr", "ms_lsqr", "ms_lsir")}}
        out["speedup_vs_fp64"] = (t64 / (dt / args.steps)) if ok else None
        del S64
    if mixed:
        # the same solve with the inner FGMRES tolerance relaxed after the first
        # refinement step (ls_iter_opts_t.inner_adapt = 1)
        Sa = L.Solver(At, b, s=s, seed=seed, terms=terms, pr=pr, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol, inner_adapt=1)
        Sa()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(args.steps):
            Sa()
        torch.cuda.synchronize()
        ta = (time.perf_counter() - t3) / args.steps
        ea = refsolve.forward_errors(Sa.x.cpu().numpy(), Sa.r.cpu().numpy(), xr, rr)
        sa = Sa.stats.as_dict()
        out["adaptive_inner"] = {"ms": 1e3 * ta, "solves_per_s": 1.0 / ta, "fwd_err_x": ea[0], "fwd_err_r": ea[1],
                                 "meets_target": ea[0] <= TARGET_ERR and ea[1] <= TARGET_ERR,
                                 "iterations": {"lsqr": sa["lsqr_its"], "lsir": sa["lsir_its"],
                                                "fgmres": sa["fgmres_its_total"]}}
        del Sa
    if not args.no_sparse and mixed:
        # the same problem with the sparse sign embedding (Section 2, zeta = 8)
        # in place of the Gaussian sketch: binary64 gather, same QR/LSQR/FGMRES
        prs = L.precs(u_s="f64", u_qr=wl["u_qr"], u=wl["u"], u_r=u_r)
        Ss = L.Solver(At, b, s=s, seed=seed, pr=prs, zeta=8, lsir_tol=lsir_tol, lsqr_tol=lsqr_tol)
        Ss()
        torch.cuda.synchronize()
        log("[bench] sparse sign embedding, 5 solves")
        t2 = time.perf_counter()
        for _ in range(5):
            Ss()
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t2) / 5
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
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(wl, P, seed, terms)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
