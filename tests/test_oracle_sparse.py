"""Pins of the oracle's sparse sign embedding (Section 2).

The pattern is checked against a scalar re-derivation from raw Philox words
(the rejection rule), its statistics against the definition (uniform distinct
rows, balanced signs, E ||Omega x||^2 = ||x||^2), the sketch against the dense
product with the explicit Omega, and the preconditioner it gives against the
paper's remark that s a small multiple of n suffices.
"""

import math

import numpy as np
import pytest

from lsdata import make_paper_problem, make_problem
from oracle import philox, qr as oqr, sketch as osk, solve as osolve


def _scalar_column(seed, prob, i, s, zeta):
    picks, signs, t = [], [], 0
    while len(picks) < zeta:
        words = philox.philox4x32_10(np.uint64(i), np.uint64(t), np.uint64(prob), np.uint64(1),
                                     seed & 0xFFFFFFFF, seed >> 32)
        for w in words:
            w = int(w)
            h = (w * s) >> 32
            if len(picks) < zeta and h not in picks:
                picks.append(h)
                signs.append(-1.0 if w & 1 else 1.0)
        t += 1
    return picks, signs


def test_pattern_follows_the_rejection_rule():
    seed, prob, m, s, zeta = (1 << 40) + 12345, 3, 300, 5, 4   # small s: many rejections
    H, S = osk.sparse_sign_pattern(seed, prob, m, s, zeta)
    for i in range(m):
        picks, signs = _scalar_column(seed, prob, i, s, zeta)
        assert list(H[i]) == picks and list(S[i]) == signs
    assert np.all(np.sort(H, axis=1)[:, 1:] != np.sort(H, axis=1)[:, :-1])   # distinct per column
    assert H.min() >= 0 and H.max() < s


def test_pattern_statistics():
    m, s, zeta = 200000, 100, 8
    H, S = osk.sparse_sign_pattern(3, 0, m, s, zeta)
    cnt = np.bincount(H.ravel(), minlength=s)
    e = m * zeta / s
    chi2 = ((cnt - e) ** 2 / e).sum()
    assert chi2 < (s - 1) + 5 * math.sqrt(2 * (s - 1))          # uniform rows
    assert abs(S.mean()) < 4 / math.sqrt(m * zeta)               # balanced signs
    assert set(np.unique(S)) == {-1.0, 1.0}


def test_sketch_equals_dense_product_and_preserves_norms():
    m, s, zeta = 700, 48, 4
    P = make_problem(m, 9, 1e2, seed=5, store="f32")
    H, S = osk.sparse_sign_pattern(11, 2, m, s, zeta)
    Om = np.zeros((s, m))
    Om[H, np.repeat(np.arange(m)[:, None], zeta, axis=1)] = S / math.sqrt(zeta)
    assert np.all(np.count_nonzero(Om, axis=0) == zeta)
    M = np.column_stack([P.A(), P.b.astype(np.float64)])
    Y = osk.sparse_sketch(P.At, P.b, s, 11, zeta, prob=2)
    assert np.max(np.abs(Y - Om @ M)) <= 1e-13 * np.max(np.abs(Om) @ np.abs(M))
    # E ||Omega x||^2 = ||x||^2: every column of Omega has unit norm
    assert np.allclose(np.linalg.norm(Om, axis=0), 1.0)
    rng = np.random.default_rng(0)
    ratios = [np.linalg.norm(Om @ x) ** 2 / np.linalg.norm(x) ** 2 for x in rng.standard_normal((300, m))]
    assert abs(np.mean(ratios) - 1.0) < 0.05


@pytest.mark.parametrize("zeta", [2, 8])
def test_sparse_sketch_preconditions_like_the_gaussian(zeta):
    # Section 2: with s a small multiple of n the sparse sign embedding gives a
    # preconditioner of the same quality (kappa(A R^-1) near 3 at s = 4n)
    for seed in (1, 2):
        P = make_paper_problem(1000, 100, 1e4, seed, store="f32")
        Y = osk.sparse_sketch(P.At, P.b, 400, seed + 100, zeta)
        R = oqr.householder_r(Y)[:100, :100]
        assert osolve.preconditioned_norms(P.At, R)[2] < 4.0


def test_sketch_rows_equal_full_sketch_rows():
    P = make_problem(3000, 11, 1e2, seed=8, store="f32")
    Y = osk.sparse_sketch(P.At, P.b, 60, 4, 4, prob=1)
    rows = [0, 17, 59]
    assert np.array_equal(osk.sparse_sketch_rows(P.At, P.b, 60, 4, 4, rows, prob=1), Y[rows])
