"""The C ABI library loads and exports every function include/ls.h declares
(CPU only: no compute call is made)."""

import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "ls.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ls_sketch", "ls_qr_r", "ls_lsqr_precond", "ls_lsir_gmres", "ls_solve",
                     "ls_workspace_size", "ls_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2410_06319_amd import _binding
    lib = _binding.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_binding.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", _binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ls_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_strerror_covers_status_codes():
    from paper_2410_06319_amd import _binding
    lib = _binding.load()
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.ls_strerror(code) and lib.ls_strerror(code) != b"unknown status"


def test_default_options_follow_section_5():
    import ctypes
    from paper_2410_06319_amd import _binding
    lib = _binding.load()
    o = _binding.IterOpts()
    lib.ls_default_iter_opts(100, _binding.FP32, ctypes.byref(o))
    assert (o.lsqr_tol, o.lsqr_maxit, o.fgmres_tol, o.fgmres_maxit, o.lsir_maxit) == (1e-6, 200, 1e-6, 50, 30)
    lib.ls_default_iter_opts(100, _binding.FP64, ctypes.byref(o))
    assert (o.lsqr_tol, o.fgmres_tol) == (1e-12, 1e-12)
    assert o.lsir_tol == pytest.approx(4 * 2.0 ** -53)


def test_struct_layouts_match_the_binding(tmp_path):
    # the header is plain C: gcc reports each field's offset and each struct's
    # size, which the ctypes mirrors in the binding must reproduce
    import ctypes
    from paper_2410_06319_amd import _binding as B
    structs = {"ls_problem_t": B.Problem, "ls_precs_t": B.Precs, "ls_sketch_opts_t": B.SketchOpts,
               "ls_iter_opts_t": B.IterOpts, "ls_stats_t": B.Stats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ls.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_sketch_plan_candidates_and_tuned_table():
    # the launch-shape candidates the library offers, and the tuned table it
    # compiles in: every entry names a known format, parts and candidate, and
    # within a (format, parts) group the cells grow in both sizes
    import paper_2410_06319_amd as L
    from paper_2410_06319_amd import _binding as B
    L.load()
    counts = {}
    for fmt in ("bf16", "f16", "e4m3", "f64"):
        k = 1
        while L.sketch_plan_info(fmt, k) is not None:
            tc, qc = L.sketch_plan_info(fmt, k)
            assert tc in (0, 128, 256, 512) and qc >= 1
            k += 1
        counts[B.PREC[fmt]] = k - 1
        assert k - 1 >= 4 and L.sketch_plan_info(fmt, 0) is None
    assert L.sketch_plan_info("bf16", 1) == (0, 4)          # plan 1: the untuned rule
    path = os.path.join(ROOT, "paper_2410_06319_amd", "csrc", "sketch_tuned.inc")
    rows = []
    for line in open(path):
        line = line.split("//")[0].strip()
        if line:
            vals = [int(v) for v in re.findall(r"-?\d+", line)]
            assert len(vals) == 5, line
            rows.append(vals)
    for fmt, terms, ncols_max, m_max, plan in rows:
        assert fmt in counts and 1 <= plan <= counts[fmt]
        assert (terms == 1) if fmt == B.FP64 else (1 <= terms <= 3)
        assert ncols_max > 0 and m_max > 0


def test_traffic_figure_follows_the_code_not_its_comments(tmp_path, monkeypatch):
    # bench.py reports the recorded HBM traffic only while the hash of the
    # pass's sources matches: comment and blank-line edits keep the hash, a
    # code edit changes it and the recorded figure is then dropped
    import sys
    sys.path.insert(0, ROOT)
    import bench
    a = tmp_path / "a.hip"
    a.write_text("int f() {\n  return 1;  // one\n}\n")
    b = tmp_path / "b.hip"
    b.write_text("// header\nint f() {\n\n  return 1;\n}  /* tail\n   comment */\n")
    c = tmp_path / "c.hip"
    c.write_text("int f() {\n  return 2;\n}\n")
    hashes = []
    for f in (a, b, c):
        monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(f)])
        hashes.append(bench.kernel_source_hash())
    assert hashes[0] == hashes[1] and hashes[0] != hashes[2]
    rec = tmp_path / "traffic.md"
    rec.write_text(f"    traffic_bytes_per_launch=2.0e+08 source_sha256_16={hashes[0]}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(b)])
    assert bench.recorded_traffic() == 2.0e8
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(c)])
    assert bench.recorded_traffic() is None
