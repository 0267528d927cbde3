"""Autotuner for the sketch's launch shape.

For a grid of problem shapes (n + 1 columns, m rows, s = 4n), sketch formats
and part counts it times every launch-shape candidate of ``ls_sketch`` (see
``ls_sketch_plan_info``: columns per block and the blocks the K-splits aim
at) on the current device, and writes the fastest per shape into
``csrc/sketch_tuned.inc``, the table the library's planner consults when
``ls_sketch_opts_t.plan`` is 0.  Rebuild the library afterwards.

A candidate replaces the default (plan 1) only when it is faster by more than
``--margin`` (default 5 %), so that timing noise does not move the table;
candidates that give the same launch for a shape are timed once.

    python -m paper_2410_06319_amd.autotune [--quick] [--out PATH] [--formats e4m3,...]

With ``--formats`` only those formats' shapes are timed; the table's rows for
the other formats are kept as they are.
"""

import argparse
import ctypes
import math
import os
import time

import torch

from . import _binding as B
from .api import precs, problem, sketch_opts, sketch_plan_info, workspace, workspace_size, iter_opts, _stream

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "csrc", "sketch_tuned.inc")

NCOLS = [33, 65, 129, 257, 501, 1001]
MROWS = [5000, 30000, 100000, 300000]
CASES = [("bf16", 1), ("bf16", 2), ("bf16", 3), ("f16", 2), ("f16", 3), ("e4m3", 2), ("e4m3", 3), ("f64", 1)]
FMT_CODE = {"bf16": B.BF16, "f16": B.FP16, "e4m3": B.FP8E4M3, "f64": B.FP64}


def plans(u_s, ncols):
    """Candidates that differ for n + 1 = ncols (a fixed width equal to the
    one the default rule picks is the same launch)."""
    out, seen, k = [], set(), 1
    while True:
        info = sketch_plan_info(u_s, k)
        if info is None:
            return out
        tc, qc = info
        if u_s != "f64" and tc == 0:
            tc = 128 if ncols <= 128 else 256 if ncols <= 256 else 512
        if (tc, qc) not in seen:
            seen.add((tc, qc))
            out.append(k)
        k += 1


def time_plan(At, b, s, u_s, terms, plan, ws, reps):
    P = problem(At, b)
    so = sketch_opts(s=s, seed=12345, terms=terms, plan=plan)
    Yt = torch.empty((P.n + 1, s), dtype=torch.float64, device=At.device)
    lib = B.load()

    def call():
        rc = lib.ls_sketch(ctypes.byref(P), ctypes.byref(so), B.PREC[u_s], Yt.data_ptr(), s, ws.data_ptr(),
                           ws.numel(), _stream())
        if rc != 0:
            raise RuntimeError(f"ls_sketch failed with status {rc}")

    call()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def bounds(grid):
    """Upper limits of the grid's cells: geometric midpoints, the last unbounded."""
    return [int(math.sqrt(a * b)) for a, b in zip(grid, grid[1:])] + [(1 << 62)]


def tune(ncols_grid, m_grid, cases, reps, margin, log):
    entries = []
    dev = torch.device("cuda")
    for u_s, terms in cases:
        for nc, nmax in zip(ncols_grid, bounds(ncols_grid)):
            cands = plans(u_s, nc)
            n = nc - 1
            for m, mmax in zip(m_grid, bounds(m_grid)):
                g = torch.Generator(device=dev).manual_seed(1000 * nc + m)
                At = torch.randn((n, m), generator=g, device=dev, dtype=torch.float32)
                b = torch.randn((m,), generator=g, device=dev, dtype=torch.float32)
                s = 4 * n
                pr = precs(u_s=u_s, u_qr="f64", u="f64", u_r="f64")
                need = 0
                for k in cands:
                    so = sketch_opts(s=s, terms=terms, plan=k)
                    need = max(need, workspace_size(problem(At, b), so, pr, iter_opts(n, "f64")))
                ws = workspace(need, dev)
                t = {k: time_plan(At, b, s, u_s, terms, k, ws, reps) for k in cands}
                best = min(t, key=t.get)
                if t[best] > (1.0 - margin) * t[1]:
                    best = 1
                log(f"{u_s} x{terms} ncols={nc} m={m}: " +
                    " ".join(f"{k}:{t[k]:.3f}" for k in cands) + f" ms -> plan {best}")
                entries.append((u_s, terms, nmax, mmax, best, t[1], t[best]))
                del At, b, ws
                torch.cuda.empty_cache()
    return entries


def kept_rows(path, formats):
    """Rows of an existing table whose format is not among `formats` (text lines, in order)."""
    if not os.path.exists(path):
        return []
    codes = {FMT_CODE[f] for f in formats}
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.rstrip("\n")
            if line.startswith("{"):
                if int(line[1:].split(",")[0]) not in codes:
                    rows.append(line)
    return rows


def write_table(entries, path, device_name, kept=()):
    lines = [f"// fmt, terms, ncols_max, m_max, plan: written by `python -m paper_2410_06319_amd.autotune`",
             f"// from ls_sketch timings on {device_name} (median of the repetitions; default",
             "// plan 1 unless another is faster by the margin).  Regenerate, then rebuild."]
    new = {}
    for u_s, terms, nmax, mmax, best, t1, tb in entries:
        new.setdefault(FMT_CODE[u_s], []).append(
            f"{{{FMT_CODE[u_s]}, {terms}, {nmax}, {mmax}, {best}}},   // {t1:.3f} -> {tb:.3f} ms")
    # kept rows and new rows grouped by format, in the order of CASES
    by_code = {}
    for line in kept:
        by_code.setdefault(int(line[1:].split(",")[0]), []).append(line)
    for code, rows in new.items():
        by_code[code] = rows
    for code in dict.fromkeys(FMT_CODE[u] for u, _ in CASES):
        lines.extend(by_code.get(code, []))
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--margin", type=float, default=0.05)
    ap.add_argument("--quick", action="store_true", help="a small grid (checks the tool, not a table to keep)")
    ap.add_argument("--formats", default="", help="comma-separated formats to retune (default: all)")
    args = ap.parse_args()
    if not torch.cuda.is_available():
        raise SystemExit("the autotuner times kernels: it needs a visible GPU")
    B.load()
    ncols, mrows, cases = NCOLS, MROWS, CASES
    if args.quick:
        ncols, mrows, cases = [33, 257], [5000, 30000], [("bf16", 2), ("f64", 1)]
    formats = [f for f in args.formats.split(",") if f]
    for f in formats:
        if f not in FMT_CODE:
            raise SystemExit(f"unknown format {f!r} (one of {', '.join(FMT_CODE)})")
    kept = []
    if formats:
        cases = [c for c in cases if c[0] in formats]
        kept = kept_rows(args.out, formats)
    t0 = time.time()
    entries = tune(ncols, mrows, cases, args.reps, args.margin, lambda s: print(s, flush=True))
    arch = getattr(torch.cuda.get_device_properties(0), "gcnArchName", "").split(":")[0]
    write_table(entries, args.out, f"{torch.cuda.get_device_name(0)} ({arch})" if arch else torch.cuda.get_device_name(0),
                kept)
    print(f"[autotune] {len(entries)} shapes in {time.time() - t0:.1f} s -> {args.out}", flush=True)


if __name__ == "__main__":
    main()
