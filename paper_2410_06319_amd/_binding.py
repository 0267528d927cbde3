"""ctypes declarations of libls's C ABI (include/ls.h).  Marshalling only."""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libls.so")

# ls_prec_t
FP64, FP32, FP16, BF16, FP8E4M3, FP64X2 = 0, 1, 2, 3, 4, 5
PREC = {"f64": FP64, "f32": FP32, "f16": FP16, "bf16": BF16, "e4m3": FP8E4M3, "f64x2": FP64X2}

# status codes
OK, NOT_CONVERGED = 0, 1
E_ARG, E_WORKSPACE, E_HIP, E_SINGULAR, E_NONFINITE, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6


class Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("store", ctypes.c_int),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("b", ctypes.c_void_p)]


class Precs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int) for k in ("u_s", "u_qr", "u", "u_r", "u_A", "u_L", "u_R")]


class SketchOpts(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int64), ("seed", ctypes.c_uint64), ("prob_id", ctypes.c_uint32),
                ("terms", ctypes.c_int32), ("col_scale", ctypes.c_int32), ("zeta", ctypes.c_int32),
                ("max_terms", ctypes.c_int32), ("plan", ctypes.c_int32), ("col_exp", ctypes.c_void_p)]


class IterOpts(ctypes.Structure):
    _fields_ = [("lsqr_tol", ctypes.c_double), ("lsqr_maxit", ctypes.c_int32),
                ("fgmres_tol", ctypes.c_double), ("fgmres_maxit", ctypes.c_int32),
                ("lsir_maxit", ctypes.c_int32), ("lsir_tol", ctypes.c_double),
                ("fallback", ctypes.c_int32), ("check_every", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("inner_adapt", ctypes.c_int32), ("x_ref", ctypes.c_void_p), ("r_ref", ctypes.c_void_p),
                ("lsqr_operand", ctypes.c_int32), ("graph", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("lsqr_its", ctypes.c_int32), ("lsir_its", ctypes.c_int32),
                ("fgmres_its_total", ctypes.c_int32), ("fallback_used", ctypes.c_int32),
                ("lsqr_normr", ctypes.c_double), ("lsqr_normar", ctypes.c_double),
                ("lsqr_normB", ctypes.c_double), ("lsir_dx_rel", ctypes.c_double),
                ("lsir_dr_rel", ctypes.c_double), ("ms_sketch", ctypes.c_double),
                ("ms_qr", ctypes.c_double), ("ms_lsqr", ctypes.c_double), ("ms_lsir", ctypes.c_double),
                ("kernel_ms", ctypes.c_double * 6), ("kernel_launches", ctypes.c_int32 * 6),
                ("kernel_work", ctypes.c_double * 6), ("sketch_terms", ctypes.c_int32),
                ("sketch_plan", ctypes.c_int32), ("kappa_est", ctypes.c_double), ("err_x", ctypes.c_double),
                ("err_r", ctypes.c_double)]

    KERNEL_CLASSES = ("sketch_mfma", "lsqr_pass", "fgmres_pass", "lsir_resid_pass", "cgs_sweep", "sparse_sketch")

    def as_dict(self):
        arrays = ("kernel_ms", "kernel_launches", "kernel_work")
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in arrays}
        for a in arrays:
            d[a] = dict(zip(self.KERNEL_CLASSES, list(getattr(self, a))))
        return d


P = ctypes.POINTER
vp = ctypes.c_void_p
i64 = ctypes.c_int64
u32 = ctypes.c_uint32

# name -> (restype, argtypes); every symbol include/ls.h declares
SIGNATURES = {
    "ls_default_iter_opts": (None, [i64, ctypes.c_int, P(IterOpts)]),
    "ls_workspace_size": (ctypes.c_int, [P(Problem), P(SketchOpts), P(Precs), P(IterOpts), P(ctypes.c_size_t)]),
    "ls_sketch": (ctypes.c_int, [P(Problem), P(SketchOpts), ctypes.c_int, vp, i64, vp, ctypes.c_size_t, vp]),
    "ls_qr_r": (ctypes.c_int, [i64, i64, ctypes.c_int, vp, i64, vp, i64, vp, ctypes.c_size_t, vp]),
    "ls_qr_workspace_size": (ctypes.c_int, [i64, i64, ctypes.c_int, P(ctypes.c_size_t)]),
    "ls_lsqr_workspace_size": (ctypes.c_int, [P(Problem), ctypes.c_int, P(IterOpts), P(ctypes.c_size_t)]),
    "ls_lsir_workspace_size": (ctypes.c_int, [P(Problem), P(Precs), P(IterOpts), P(ctypes.c_size_t)]),
    "ls_qr_r_noalloc": (ctypes.c_int, [i64, i64, ctypes.c_int, vp, i64, vp, i64, vp]),
    "ls_lsqr_precond": (ctypes.c_int, [P(Problem), vp, i64, ctypes.c_int, vp, P(IterOpts), P(Stats), vp,
                                       ctypes.c_size_t, vp]),
    "ls_lsir_gmres": (ctypes.c_int, [P(Problem), vp, i64, P(Precs), vp, vp, ctypes.c_int, P(IterOpts), P(Stats),
                                     vp, ctypes.c_size_t, vp]),
    "ls_solve": (ctypes.c_int, [P(Problem), P(SketchOpts), P(Precs), P(IterOpts), vp, vp, P(Stats), vp,
                                ctypes.c_size_t, vp]),
    "ls_omega": (ctypes.c_int, [ctypes.c_uint64, u32, i64, i64, ctypes.c_int, vp, i64, vp]),
    "ls_philox": (ctypes.c_int, [u32, u32, u32, u32, u32, u32, i64, vp, vp]),
    "ls_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ls_sketch_terms_for": (ctypes.c_int, [ctypes.c_double, ctypes.c_int, ctypes.c_int32, ctypes.c_int32]),
    "ls_sketch_split_rows": (ctypes.c_int, [P(Problem), P(SketchOpts), ctypes.c_int, P(ctypes.c_int64)]),
    "ls_sketch_plan_info": (ctypes.c_int, [ctypes.c_int, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]),
    "ls_workspace_size_batched": (ctypes.c_int, [ctypes.c_int, P(Problem), P(SketchOpts), P(Precs), P(IterOpts),
                                                 ctypes.c_int, P(ctypes.c_size_t)]),
    "ls_solve_batched": (ctypes.c_int, [ctypes.c_int, P(Problem), P(SketchOpts), P(Precs), P(IterOpts),
                                        P(ctypes.c_void_p), P(ctypes.c_void_p), P(Stats), ctypes.c_int, vp,
                                        ctypes.c_size_t, vp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libls.so (built in-tree by paper_2410_06319_amd.build); raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libls.so is not built ({path}); run python -m paper_2410_06319_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LsError(RuntimeError):
    def __init__(self, code, where):
        msg = load().ls_strerror(code).decode()
        super().__init__(f"{where}: status {code} ({msg})")
        self.code = code
