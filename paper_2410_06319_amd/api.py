"""Python entry points over libls (same names as the C ABI).

torch supplies device memory and the current HIP stream; every step of the
method runs in libls's kernels.  Arrays use the library's layout: A is passed
as ``At`` of shape (n, m) (the column-major m x n matrix, lda = At.stride(0)),
vectors as 1-D tensors.
"""

import ctypes

import torch

from . import _binding as B


def _dev_check(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("libls works on device tensors; got a CPU tensor")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _store_code(dtype):
    if dtype == torch.float32:
        return B.FP32
    if dtype == torch.float64:
        return B.FP64
    raise ValueError(f"A and b must be float32 or float64, got {dtype}")


def problem(At: torch.Tensor, b: torch.Tensor) -> B.Problem:
    _dev_check(At, b)
    if At.dim() != 2 or At.stride(1) != 1 or b.dim() != 1 or b.stride(0) != 1:
        raise ValueError("At must be (n, m) with unit stride along m; b must be contiguous")
    if At.dtype != b.dtype:
        raise ValueError("A and b must share a storage precision")
    n, m = At.shape
    if b.shape[0] != m:
        raise ValueError("b must have m entries")
    return B.Problem(m=m, n=n, store=_store_code(At.dtype), A=At.data_ptr(), lda=At.stride(0), b=b.data_ptr())


def precs(u_s="bf16", u_qr="f32", u="f32", u_r="f64", u_A=None, u_L=None, u_R=None) -> B.Precs:
    u_A = u_A or u
    return B.Precs(u_s=B.PREC[u_s], u_qr=B.PREC[u_qr], u=B.PREC[u], u_r=B.PREC[u_r],
                   u_A=B.PREC[u_A], u_L=B.PREC[u_L or u_A], u_R=B.PREC[u_R or u_A])


def sketch_opts(s=0, seed=0, prob_id=0, terms=1, col_scale=0, zeta=0, max_terms=0, plan=0, col_exp=None) -> B.SketchOpts:
    return B.SketchOpts(s=s, seed=seed, prob_id=prob_id, terms=terms, col_scale=col_scale, zeta=zeta,
                        max_terms=max_terms, plan=plan, col_exp=col_exp)


def iter_opts(n, u="f32", **kw) -> B.IterOpts:
    o = B.IterOpts()
    B.load().ls_default_iter_opts(n, B.PREC[u], ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _check(rc, where, allow_not_converged=True):
    if rc < 0 or (rc == B.NOT_CONVERGED and not allow_not_converged):
        raise B.LsError(rc, where)
    return rc


def workspace(nbytes: int, device=None) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def workspace_size(P, so, pr, io) -> int:
    n = ctypes.c_size_t(0)
    _check(B.load().ls_workspace_size(ctypes.byref(P), ctypes.byref(so), ctypes.byref(pr), ctypes.byref(io),
                                      ctypes.byref(n)), "ls_workspace_size")
    return n.value


def qr_workspace_size(s, ncols, u_qr="f32") -> int:
    n = ctypes.c_size_t(0)
    _check(B.load().ls_qr_workspace_size(int(s), int(ncols), B.PREC[u_qr], ctypes.byref(n)), "ls_qr_workspace_size")
    return n.value


def ls_sketch(At, b, s, seed=0, u_s="bf16", terms=1, prob_id=0, col_scale=0, zeta=0, ws=None, plan=0,
              col_exp=None):
    """Y = Omega [A b] (s x (n+1), float64; returned as a (n+1, s) tensor = column-major Y).

    u_s: "f64", "bf16", "f16" or "e4m3"; col_scale 0 = automatic (on for f16 and e4m3);
    col_exp: optional int32 device tensor of n+1 entries receiving the column exponents."""
    P = problem(At, b)
    so = sketch_opts(s=s, seed=seed, prob_id=prob_id, terms=terms, col_scale=col_scale, zeta=zeta, plan=plan,
                     col_exp=None if col_exp is None else col_exp.data_ptr())
    pr = precs(u_s=u_s, u_qr="f64", u="f64", u_r="f64")
    if ws is None:
        ws = workspace(workspace_size(P, so, pr, iter_opts(P.n, "f64")), At.device)
    Yt = torch.empty((P.n + 1, s), dtype=torch.float64, device=At.device)
    _check(B.load().ls_sketch(ctypes.byref(P), ctypes.byref(so), B.PREC[u_s], Yt.data_ptr(), s, ws.data_ptr(),
                              ws.numel(), _stream()), "ls_sketch")
    return Yt


def ls_qr_r(Yt: torch.Tensor, u_qr="f32", ws=None):
    """R factor (ncols x ncols, diag > 0) of Y given as Yt (ncols, s) float64 (left unchanged).

    Returns Rt (ncols, ncols) = the column-major R, i.e. R = Rt.T.
    """
    _dev_check(Yt)
    ncols, s = Yt.shape
    if Yt.dtype != torch.float64 or Yt.stride(1) != 1:
        raise ValueError("Yt must be float64 with unit stride along s")
    if ws is None:
        ws = workspace(qr_workspace_size(s, ncols, u_qr), Yt.device)
    Rt = torch.empty((ncols, ncols), dtype=torch.float64, device=Yt.device)
    _check(B.load().ls_qr_r(s, ncols, B.PREC[u_qr], Yt.data_ptr(), Yt.stride(0), Rt.data_ptr(), ncols,
                            ws.data_ptr(), ws.numel(), _stream()), "ls_qr_r")
    return Rt


def ls_lsqr_precond(At, b, Rt, x, u="f32", ws=None, **opts):
    """Preconditioned LSQR from x (float64 (n,), updated in place).  Rt: (n, n) column-major R."""
    P = problem(At, b)
    io = iter_opts(P.n, u, **opts)
    st = B.Stats()
    if ws is None:
        nbytes = ctypes.c_size_t(0)
        _check(B.load().ls_lsqr_workspace_size(ctypes.byref(P), B.PREC[u], ctypes.byref(io), ctypes.byref(nbytes)),
               "ls_lsqr_workspace_size")
        ws = workspace(nbytes.value, At.device)
    rc = B.load().ls_lsqr_precond(ctypes.byref(P), Rt.data_ptr(), Rt.stride(0), B.PREC[u], x.data_ptr(),
                                  ctypes.byref(io), ctypes.byref(st), ws.data_ptr(), ws.numel(), _stream())
    _check(rc, "ls_lsqr_precond")
    return rc, st.as_dict()


def ls_lsir_gmres(At, b, Rt, x, r, pr=None, r_given=False, ws=None, **opts):
    """Refinement (Algorithm 2's refinement loop); x (n,) and r (m,) float64, updated in place."""
    P = problem(At, b)
    pr = pr or precs()
    io = iter_opts(P.n, "f64" if pr.u == B.FP64 else "f32", **opts)
    st = B.Stats()
    if ws is None:
        nbytes = ctypes.c_size_t(0)
        _check(B.load().ls_lsir_workspace_size(ctypes.byref(P), ctypes.byref(pr), ctypes.byref(io),
                                               ctypes.byref(nbytes)), "ls_lsir_workspace_size")
        ws = workspace(nbytes.value, At.device)
    rc = B.load().ls_lsir_gmres(ctypes.byref(P), Rt.data_ptr(), Rt.stride(0), ctypes.byref(pr), x.data_ptr(),
                                r.data_ptr(), int(r_given), ctypes.byref(io), ctypes.byref(st), ws.data_ptr(),
                                ws.numel(), _stream())
    _check(rc, "ls_lsir_gmres")
    return rc, st.as_dict()


class Solver:
    """Reusable ls_solve call: holds the options and one workspace for a problem shape."""

    def __init__(self, At, b, s=0, seed=0, prob_id=0, terms=1, pr=None, col_scale=0, zeta=0, max_terms=0, **opts):
        self.P = problem(At, b)
        self.At, self.b = At, b
        self.so = sketch_opts(s=s, seed=seed, prob_id=prob_id, terms=terms, col_scale=col_scale, zeta=zeta,
                              max_terms=max_terms)
        self.pr = pr or precs()
        self.io = iter_opts(self.P.n, "f64" if self.pr.u == B.FP64 else "f32", **opts)
        self.ws = workspace(workspace_size(self.P, self.so, self.pr, self.io), At.device)
        self.x = torch.empty(self.P.n, dtype=torch.float64, device=At.device)
        self.r = torch.empty(self.P.m, dtype=torch.float64, device=At.device)
        self.stats = B.Stats()

    def __call__(self, check=True):
        rc = B.load().ls_solve(ctypes.byref(self.P), ctypes.byref(self.so), ctypes.byref(self.pr),
                               ctypes.byref(self.io), self.x.data_ptr(), self.r.data_ptr(),
                               ctypes.byref(self.stats), self.ws.data_ptr(), self.ws.numel(), _stream())
        if check:
            _check(rc, "ls_solve")
        return rc


def ls_solve(At, b, s=0, seed=0, terms=1, pr=None, col_scale=0, prob_id=0, zeta=0, max_terms=0, **opts):
    """The whole method.  Returns (x, r, status, stats dict); zeta > 0 selects the sparse sign embedding;
    max_terms > terms lets the solve add sketch parts while kappa_est u_s^terms > 1."""
    S = Solver(At, b, s=s, seed=seed, prob_id=prob_id, terms=terms, pr=pr, col_scale=col_scale, zeta=zeta,
               max_terms=max_terms, **opts)
    rc = S()
    return S.x, S.r, rc, S.stats.as_dict()


def ls_solve_batched(problems, s=0, seeds=None, terms=1, pr=None, col_scale=0, nworkers=0, max_terms=0, **opts):
    """The whole method for a list of (At, b) problems on one device.

    Returns (xs, rs, status, list of stats dicts); s = 0 uses 4 n per problem.
    """
    nprob = len(problems)
    Ps = (B.Problem * nprob)(*[problem(At, b) for At, b in problems])
    seeds = seeds if seeds is not None else [0] * nprob
    sos = (B.SketchOpts * nprob)(*[sketch_opts(s=s, seed=seeds[i], prob_id=i, terms=terms, col_scale=col_scale,
                                               max_terms=max_terms)
                                   for i in range(nprob)])
    pr = pr or precs()
    io = iter_opts(max(p.n for p in Ps), "f64" if pr.u == B.FP64 else "f32", **opts)
    # the LSQR limit 2n is per problem (Section 5): zero lets the library take each problem's own
    if "lsqr_maxit" not in opts:
        io.lsqr_maxit = 0
    nbytes = ctypes.c_size_t(0)
    _check(B.load().ls_workspace_size_batched(nprob, Ps, sos, ctypes.byref(pr), ctypes.byref(io), nworkers,
                                              ctypes.byref(nbytes)), "ls_workspace_size_batched")
    dev = problems[0][0].device
    ws = workspace(nbytes.value, dev)
    xs = [torch.empty(Ps[i].n, dtype=torch.float64, device=dev) for i in range(nprob)]
    rs = [torch.empty(Ps[i].m, dtype=torch.float64, device=dev) for i in range(nprob)]
    xp = (ctypes.c_void_p * nprob)(*[t.data_ptr() for t in xs])
    rp = (ctypes.c_void_p * nprob)(*[t.data_ptr() for t in rs])
    stats = (B.Stats * nprob)()
    rc = B.load().ls_solve_batched(nprob, Ps, sos, ctypes.byref(pr), ctypes.byref(io), xp, rp, stats, nworkers,
                                   ws.data_ptr(), ws.numel(), _stream())
    _check(rc, "ls_solve_batched")
    return xs, rs, rc, [stats[i].as_dict() for i in range(nprob)]


def sketch_plan_info(u_s, plan):
    """(columns per block, target blocks in quarters of the compute units) of
    launch shape ``plan`` of the sketch in ``u_s``, or None past the last one."""
    tc, qc = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = B.load().ls_sketch_plan_info(B.PREC[u_s], int(plan), ctypes.byref(tc), ctypes.byref(qc))
    return (tc.value, qc.value) if rc == 0 else None


def sketch_split_rows(At, b, s, u_s="bf16", terms=1, plan=0, prob_id=0, col_scale=0, zeta=0):
    """Rows of [A b] each binary32 partial sum of the sketch covers (its K-split length)."""
    P = problem(At, b)
    so = sketch_opts(s=s, terms=terms, plan=plan, prob_id=prob_id, col_scale=col_scale, zeta=zeta)
    rows = ctypes.c_int64(0)
    _check(B.load().ls_sketch_split_rows(ctypes.byref(P), ctypes.byref(so), B.PREC[u_s], ctypes.byref(rows)),
           "ls_sketch_split_rows")
    return rows.value


def sketch_terms_for(kappa_est, u_s="bf16", terms=1, max_terms=3):
    """Parts the solve sketches with next after an R formed with ``terms`` parts (host only)."""
    return B.load().ls_sketch_terms_for(float(kappa_est), B.PREC[u_s], int(terms), int(max_terms))


def ls_omega(seed, s, m, fmt="bf16", prob_id=0, device="cuda"):
    """Unscaled sketch operator S (s x m) as used by the sketch in ``fmt``; returned as (m, s) = column-major S."""
    St = torch.empty((m, s), dtype=torch.float64, device=device)
    _check(B.load().ls_omega(seed, prob_id, s, m, B.PREC[fmt], St.data_ptr(), s, _stream()), "ls_omega")
    return St


def ls_philox(c0, c1, c2, c3, k0, k1, count, device="cuda"):
    """Philox4x32-10 blocks for counters (c0 + t, c1, c2, c3), t < count: (count, 4) int64 tensor of words."""
    out = torch.empty(4 * count, dtype=torch.int32, device=device)
    _check(B.load().ls_philox(c0, c1, c2, c3, k0, k1, count, out.data_ptr(), _stream()), "ls_philox")
    return out.view(count, 4).to(torch.int64) & 0xFFFFFFFF
