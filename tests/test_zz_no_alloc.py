"""ls_qr_r_noalloc: Algorithm 1's QR with its scratch in the library's static
device array, against ls_qr_r (same kernels, caller workspace) through the C
ABI.  Both run the same kernels on the same input, so R must agree bit for
bit; two calls in a row, the second smaller, show that the contents the
first call leaves in the shared array do not leak into the second."""

import ctypes

import numpy as np
import pytest
import torch

from lsdata import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2410_06319_amd import _binding
    _binding.load()
    return _binding


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _qr_pair(B, Y, u_qr):
    """R from ls_qr_r (workspace from torch) and from ls_qr_r_noalloc."""
    lib = B.load()
    s, ncols = Y.shape
    Yt = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()
    prec = B.PREC[u_qr]
    ws_bytes = ctypes.c_size_t(0)
    assert lib.ls_qr_workspace_size(s, ncols, prec, ctypes.byref(ws_bytes)) == 0
    ws = torch.empty(ws_bytes.value, dtype=torch.uint8, device="cuda")
    R1 = torch.full((ncols, ncols), np.nan, dtype=torch.float64, device="cuda")
    R2 = torch.full((ncols, ncols), np.nan, dtype=torch.float64, device="cuda")
    rc1 = lib.ls_qr_r(s, ncols, prec, Yt.data_ptr(), s, R1.data_ptr(), ncols, ws.data_ptr(), ws.numel(), _stream())
    rc2 = lib.ls_qr_r_noalloc(s, ncols, prec, Yt.data_ptr(), s, R2.data_ptr(), ncols, _stream())
    torch.cuda.synchronize()
    return rc1, rc2, R1.cpu().numpy().T, R2.cpu().numpy().T


@pytest.mark.parametrize("u_qr", ["f32", "f64"])
def test_noalloc_qr_equals_workspace_qr_on_two_calls(B, u_qr):
    # first a 2000 x 501 sketch-shaped matrix, then a smaller, ragged 777 x 45
    for k, (s, ncols) in enumerate([(2000, 501), (777, 45)]):
        Y = make_problem(s, ncols, 1e3, seed=40 + k, store="f64").A()
        print(f"noalloc QR {u_qr} call {k}: {s} x {ncols}", flush=True)
        rc1, rc2, R1, R2 = _qr_pair(B, Y, u_qr)
        assert rc1 == 0 and rc2 == 0
        assert np.all(np.diag(R2) > 0) and np.all(np.tril(R2, -1) == 0)
        assert np.array_equal(R1, R2)


def test_noalloc_qr_reports_rank_deficiency_after_a_good_call(B):
    # the flag word in the shared array starts at zero on every call: a good
    # call after a rank-deficient one succeeds again
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((300, 12))
    Y[:, 5] = 0.0
    rc1, rc2, _, _ = _qr_pair(B, Y, "f64")
    assert rc1 == B.E_SINGULAR and rc2 == B.E_SINGULAR
    Y[:, 5] = rng.standard_normal(300)
    rc1, rc2, R1, R2 = _qr_pair(B, Y, "f64")
    assert rc1 == 0 and rc2 == 0 and np.array_equal(R1, R2)


def test_noalloc_qr_rejects_shapes_beyond_its_scratch(B):
    # 8192 x 2049 in binary64 needs about 134 MB of scratch, beyond the
    # array: refused before anything reaches the device
    lib = B.load()
    Yt = torch.zeros(16, dtype=torch.float64, device="cuda")
    R = torch.zeros(16, dtype=torch.float64, device="cuda")
    rc = lib.ls_qr_r_noalloc(8192, 2049, B.FP64, Yt.data_ptr(), 8192, R.data_ptr(), 2049, _stream())
    assert rc == B.E_WORKSPACE
