"""Pins of the condition estimate and the parts rule (Section 4's condition
kappa(A) u_s < 1 for a multi-part narrow sketch), and the library's host rule
against the oracle's.

kappa_est is pinned by closed forms (diagonal and scaled identity factors)
and by the bounds kappa_2 / sqrt(n) <= kappa_est <= sqrt(n) kappa_2 against
an SVD; the parts rule by its boundary values, where kappa u^terms crosses 1.
"""

import math

import numpy as np
import pytest

from lsdata import make_paper_problem
from oracle import qr as oqr, sketch as osk, solve as osolve


def test_kappa_est_diagonal_closed_form():
    d = np.array([1.0, 0.5, 1e-3, 4.0])
    want = math.sqrt(np.sum(d ** 2)) * math.sqrt(np.sum(d ** -2.0)) / 2.0
    assert osolve.kappa_est(np.diag(d)) == pytest.approx(want, rel=1e-14)
    assert osolve.kappa_est(3.0 * np.eye(25)) == pytest.approx(5.0, rel=1e-14)


def test_kappa_est_lies_within_sqrt_n_of_kappa_2():
    rng = np.random.default_rng(4)
    for n in (2, 10, 60):
        for scale in (1.0, 1e3):
            R = np.triu(rng.standard_normal((n, n))) + np.diag(rng.uniform(0.1, 1.0, n) * scale)
            k2 = np.linalg.cond(R)
            ke = osolve.kappa_est(R)
            assert k2 / math.sqrt(n) * (1 - 1e-12) <= ke <= math.sqrt(n) * k2 * (1 + 1e-12)


def test_kappa_est_tracks_kappa_a_on_the_paper_problem():
    # geometric singular values: kappa_est of the sketch's R stays within a
    # small factor of kappa(A) (the embedding distorts by about 3 at s = 4n)
    for kappa in (1e2, 1e4):
        P = make_paper_problem(1000, 100, kappa, 1, store="f32")
        Y, _ = osk.sketch(P.At, P.b, 400, 101, fmt="f64")
        R = oqr.householder_r(Y)[:100, :100]
        assert kappa / 5 < osolve.kappa_est(R) < 5 * kappa


@pytest.mark.parametrize("fmt,bits", [("bf16", 8), ("f16", 11), ("e4m3", 4)])
def test_terms_rule_boundaries(fmt, bits):
    u = 2.0 ** -bits
    below, above = (1 - 1e-9) / u, (1 + 1e-9) / u
    assert osolve.terms_for(below, fmt, 1, 3) == 1
    assert osolve.terms_for(above, fmt, 1, 3) == 2
    assert osolve.terms_for(below / u, fmt, 2, 3) == 2
    assert osolve.terms_for(above / u, fmt, 2, 3) == 3
    assert osolve.terms_for(1e30, fmt, 3, 3) == 3       # at most max_terms
    assert osolve.terms_for(1e30, fmt, 1, 1) == 1       # rule off
    assert osolve.terms_for(float("inf"), fmt, 1, 2) == 2


def test_terms_rule_binary64_has_one_part():
    assert osolve.terms_for(1e30, "f64", 1, 3) == 1


def test_library_rule_equals_oracle_rule():
    import paper_2410_06319_amd as L
    L.load()
    for fmt in ("bf16", "f16", "e4m3", "f64"):
        for kappa in (1.0, 10.0, 255.0, 257.0, 2047.0, 2049.0, 15.0, 17.0, 6.5e4, 6.6e4, 1e6, 1e12,
                      float("inf"), float("nan")):
            for terms in (1, 2, 3, 4, 5):
                for max_terms in (0, 1, 2, 3, 4, 5):
                    want = osolve.terms_for(kappa, fmt, terms, max_terms)
                    got = L.sketch_terms_for(kappa, fmt, terms, max_terms)
                    assert got == want, (fmt, kappa, terms, max_terms)


def test_oracle_solve_adds_parts_until_the_condition_holds():
    # kappa(A) = 1e4, bf16: one part leaves kappa u_s near 40, two parts 0.15
    P = make_paper_problem(1000, 100, 1e4, 2, store="f32")
    _, _, info = osolve.solve(P.At, P.b, 400, 102, fmt="bf16", terms=1, max_terms=3, lsqr_tol=1e-6,
                              lsir_tol=4 * 2.0 ** -24, fgmres_tol=1e-6, u_r="f64")
    assert info["terms"] == 2
