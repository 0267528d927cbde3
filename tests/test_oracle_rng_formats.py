"""Pins of the oracle's random stream and format emulation (CPU only)."""

import math

import numpy as np
import pytest
import torch
from scipy import stats

from conftest import read_golden
from oracle import formats, philox
from oracle import sketch as osketch


def test_philox_known_answer_vectors():
    for row in read_golden("philox4x32_10_kat.txt"):
        v = [int(t, 16) for t in row]
        out = philox.philox4x32_10(*v[0:4], v[4], v[5])
        assert [int(o) for o in out] == v[6:10]


def test_philox_counter_words_all_matter():
    base = [int(x) for x in philox.philox4x32_10(1, 2, 3, 4, 5, 6)]
    for pos in range(4):
        c = [1, 2, 3, 4]
        c[pos] ^= 1
        assert [int(x) for x in philox.philox4x32_10(*c, 5, 6)] != base
    assert [int(x) for x in philox.philox4x32_10(1, 2, 3, 4, 5 ^ 1, 6)] != base
    assert [int(x) for x in philox.philox4x32_10(1, 2, 3, 4, 5, 6 ^ 1)] != base


def test_philox_vectorised_matches_scalar():
    c0 = np.arange(50, dtype=np.uint64)
    out = philox.philox4x32_10(c0, 7, 9, 0, 0x1234, 0x5678)
    for i in (0, 17, 49):
        one = philox.philox4x32_10(i, 7, 9, 0, 0x1234, 0x5678)
        assert [int(o[i]) for o in out] == [int(x) for x in one]


def test_uniform_from_word_exact_and_open_interval():
    w = np.array([0, 1, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    u = philox.uniform_from_word(w)
    assert u[0] == 2.0 ** -24 and u[2] == 2.0 ** -24 and u[3] == 3 * 2.0 ** -24
    assert u[4] == 1.0 - 2.0 ** -24
    assert u[5] == 0.5 + 2.0 ** -24
    assert np.all((u > 0) & (u < 1))
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_box_muller_special_values():
    z0, z1 = philox.box_muller(np.exp(-0.5), 0.0)          # radius 1, angle 0
    assert abs(z0 - 1.0) < 1e-15 and abs(z1) < 1e-15
    z0, z1 = philox.box_muller(np.exp(-2.0), 0.25)         # radius 2, angle pi/2
    assert abs(z0) < 1e-15 and abs(z1 - 2.0) < 1e-15
    z0, z1 = philox.box_muller(np.exp(-0.5), 0.5)
    assert abs(z0 + 1.0) < 1e-15


def test_gaussian_block_distribution():
    z = philox.gaussian_block(seed=2410063190, prob=0, k0=0, k1=64, i0=0, i1=4096).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2 / n)
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 5 * math.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two members of a Box-Muller pair and neighbouring blocks are uncorrelated
    zz = philox.gaussian_block(2410063190, 0, 0, 256, 0, 1024)
    for a, b in ((0, 1), (1, 2), (0, 4), (3, 4)):
        corr = np.corrcoef(zz[:, a::8].ravel(), zz[:, b::8].ravel())[0, 1]
        assert abs(corr) < 5 / math.sqrt(zz[:, a::8].size)


def test_gaussian_block_windows_agree():
    full = philox.gaussian_block(7, 3, 0, 10, 0, 37)
    part = philox.gaussian_block(7, 3, 2, 9, 5, 30)
    assert np.array_equal(part, full[2:9, 5:30])
    other = philox.gaussian_block(7, 4, 0, 10, 0, 37)        # another problem id
    assert not np.allclose(full, other)


def _torch_round(x, dtype):
    return torch.from_numpy(x.astype(np.float32)).to(dtype).to(torch.float64).numpy()


@pytest.mark.parametrize("fmt,dtype", [("bf16", torch.bfloat16), ("f16", torch.float16),
                                       ("e4m3", torch.float8_e4m3fn)])
def test_round_to_matches_torch_casts(fmt, dtype):
    rng = np.random.default_rng(3)
    bits = rng.integers(0, 2 ** 32, 400_000, dtype=np.uint64).astype(np.uint32)
    with np.errstate(invalid="ignore"):
        x = bits.view(np.float32).astype(np.float64)
    fmax = formats.FORMATS[fmt][2]
    keep = np.isfinite(x) & (np.abs(x) <= fmax)
    # also every value near the format's grid and its subnormal range
    t, emin, _ = formats.FORMATS[fmt]
    grid = np.ldexp(rng.integers(1, 2 ** (t + 1), 20000).astype(np.float64), rng.integers(emin - t - 3, 8, 20000))
    grid = np.concatenate([grid, grid * (1 + 2.0 ** -(t + 1)), -grid])
    x = np.concatenate([x[keep], grid[np.abs(grid) <= fmax]]).astype(np.float32).astype(np.float64)
    ours = formats.round_to(x, fmt)
    ref = _torch_round(x, dtype)
    assert np.array_equal(ours, ref)


def test_e4m3_saturates():
    assert formats.round_to(np.array([460.0, 1e6, -1e6]), "e4m3").tolist() == [448.0, 448.0, -448.0]


def test_column_exponents_are_largest_safe_powers_of_two():
    rng = np.random.default_rng(5)
    M = rng.standard_normal((100, 7)) * np.ldexp(1.0, rng.integers(-30, 30, 7))[None, :]
    M[:, 3] = 0.0
    for fmt in ("f16", "e4m3"):
        e = formats.column_exponents(M, fmt)
        fmax = formats.FORMATS[fmt][2]
        for j in range(7):
            mx = np.abs(M[:, j]).max()
            if mx == 0:
                assert e[j] == 0
                continue
            assert mx * 2.0 ** e[j] <= fmax < mx * 2.0 ** (e[j] + 1)
    assert np.all(formats.column_exponents(M, "bf16") == 0)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
def test_split_terms_error_shrinks_geometrically(fmt):
    rng = np.random.default_rng(9)
    M = rng.uniform(0.5, 1.0, 4000) * rng.choice([-1, 1], 4000)
    u = formats.UNIT_ROUNDOFF[fmt]
    for terms in (1, 2):
        T = formats.split_terms(M, fmt, terms)
        for t in T:
            assert np.array_equal(formats.round_to(t, fmt), t)
        err = np.max(np.abs(np.sum(T, axis=0) - M) / np.abs(M))
        assert err <= u ** terms * 2.0 + 1e-300


# ------------------------------------------------------------------ narrow-format sketch entries
def test_normal_quantiles16_against_mpmath():
    # z[U] = Phi^-1((U + 1/2) / 2^16): compared with mpmath's inverse error
    # function at 40 digits (an independent evaluation), increasing and odd
    mpmath = pytest.importorskip("mpmath")
    z = philox.normal_quantiles16()
    assert z.shape == (65536,)
    assert np.all(np.diff(z) > 0)
    assert np.array_equal(z[::-1], -z)
    mpmath.mp.dps = 40
    for U in list(range(0, 65536, 611)) + [0, 1, 2, 32767, 32768, 65534, 65535]:
        p = mpmath.mpf(2 * U + 1) / 131072
        ref = float(mpmath.sqrt(2) * mpmath.erfinv(2 * p - 1))
        assert abs(z[U] - ref) <= 1e-15 * max(1.0, abs(ref)), U


def test_normal_quantiles16_distribution():
    z = philox.normal_quantiles16()
    U = np.arange(65536)
    # the normal distribution function (ndtr, another routine) maps them back
    assert np.max(np.abs(stats.norm.cdf(z) - (U + 0.5) / 65536)) < 1e-13
    assert abs(z.sum()) < 1e-9
    v = np.mean(z * z)          # the law's tails end near 4.32: slightly under 1
    assert 0.9999 < v < 1.0
    assert 4.32 < z[-1] < 4.33


def test_uniform16_stream():
    seed, prob = 2410063190, 3
    U = philox.uniform16_block(seed, prob, 0, 5, 0, 40)
    # entry (k, i): half i % 2 of word (i % 8) // 2 of the block (i // 8, k, prob, 2)
    for k, i in ((0, 0), (0, 1), (0, 7), (2, 13), (4, 39)):
        w = philox.philox4x32_10(i // 8, k, prob, 2, seed & 0xFFFFFFFF, seed >> 32)
        assert U[k, i] == (int(w[(i % 8) // 2]) >> (16 * (i % 2))) & 0xFFFF
    part = philox.uniform16_block(seed, prob, 1, 4, 3, 29)
    assert np.array_equal(part, U[1:4, 3:29])
    big = philox.uniform16_block(seed, prob, 0, 64, 0, 4096)
    counts = np.bincount((big >> 8).ravel(), minlength=256)
    assert stats.chisquare(counts).pvalue > 1e-4
    for a, b in ((0, 1), (1, 2), (3, 4), (7, 8)):
        corr = np.corrcoef(big[:, a::16].ravel(), big[:, b::16].ravel())[0, 1]
        assert abs(corr) < 5 / math.sqrt(big[:, a::16].size)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
def test_format_quantiles_round_far_from_ties(fmt):
    # any evaluation of z within 1e-12 relative rounds to the same format value
    z = philox.normal_quantiles16()
    lo = formats.round_to(z * (1 - 1e-12), fmt)
    hi = formats.round_to(z * (1 + 1e-12), fmt)
    assert np.array_equal(lo, hi)
    q = osketch.format_quantiles(fmt)
    assert np.array_equal(q, formats.round_to(z, fmt))
    assert np.array_equal(q[::-1], -q)


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_narrow_sketch_entries_moments(fmt):
    # sample moments of S against the exact moments of the 2^16 rounded quantiles
    q = osketch.format_quantiles(fmt)
    m2, m4 = np.mean(q ** 2), np.mean(q ** 4)
    S = osketch.quantised_gaussian_block(11, 0, 0, 64, 0, 4096, fmt).ravel()
    n = S.size
    assert abs(S.mean()) < 5 * math.sqrt(m2 / n)
    assert abs(np.mean(S ** 2) - m2) < 5 * math.sqrt((m4 - m2 ** 2) / n)
    assert abs(m2 - 1.0) < (2e-2 if fmt == "e4m3" else 2e-3)
