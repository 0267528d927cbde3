"""Philox4x32-10 and the Gaussian sketch stream (oracle, test use only).

Philox4x32-10 follows Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter and a 2 x 32-bit
key; each of the ten rounds multiplies counter words 0 and 2 by the two
Philox multipliers, keeps the high and low halves of the 64-bit products,
XORs the high halves with the other two counter words and the round key, and
permutes; the key is advanced by the two Weyl constants between rounds.

Gaussian entries of Omega (Section 2: entries N(0, 1/s); Section 5:
Omega = (4n)^(-1/2) G with G standard normal).  The paper leaves the random
number generator open; it is fixed here as follows.  Key (seed mod 2^32,
seed div 2^32); entry S[k, i] is row k < s of the sketch, column i < m (the
column that multiplies row i of A), of problem ``prob``.

Binary64 sketch (``gaussian_block``):
* S[k, i] comes from the Philox block with counter (i // 4, k, prob, 0).
* Its four words w0..w3 give four uniforms u = (2 * (w >> 9) + 1) * 2^-24,
  which are exact in binary32 and lie in (0, 1).
* Box-Muller: (u0, u1) -> sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1) give
  columns 4q and 4q+1, (u2, u3) give columns 4q+2 and 4q+3.

Narrow-format sketches (bf16, fp16, e4m3; ``uniform16_block``,
``normal_quantiles16``):
* S[k, i] comes from the Philox block with counter (i // 8, k, prob, 2): its
  16-bit uniform U is bits 16 (i mod 2) .. 16 (i mod 2) + 15 of word
  (i mod 8) // 2 (eight entries per block);
* S[k, i] = Phi^-1((U + 1/2) / 2^16), the midpoint quantile of the standard
  normal law, then rounded to the format.  The entry is a Gaussian drawn to
  16-bit resolution (its tails end at about 4.3); the format keeps fewer bits
  than that resolution over most of the range (e4m3 everywhere, bf16 outside
  |z| < 0.01).

Omega = S / sqrt(s); the 1/sqrt(s) is applied after the product.
"""

import numpy as np
from scipy.special import ndtri

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on (broadcastable) uint32 counters with key (k0, k1).

    Returns four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for rnd in range(10):
        if rnd > 0:
            k0 = np.uint64((int(k0) + PHILOX_W0) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + PHILOX_W1) & 0xFFFFFFFF)
        p0 = m0 * c0                      # < 2^64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def uniform_from_word(w):
    """u = (2 * (w >> 9) + 1) * 2^-24, exact in binary32 and binary64."""
    w = np.asarray(w, dtype=np.uint32)
    return ((w >> np.uint32(9)).astype(np.float64) * 2.0 + 1.0) * 2.0 ** -24


def box_muller(u0, u1):
    """Pair of independent standard normals from two uniforms in (0, 1), float64."""
    rad = np.sqrt(-2.0 * np.log(u0))
    ang = 2.0 * np.pi * u1
    return rad * np.cos(ang), rad * np.sin(ang)


def gaussian_block(seed: int, prob: int, k0: int, k1: int, i0: int, i1: int) -> np.ndarray:
    """Unscaled Gaussian entries S[k, i], k in [k0, k1), i in [i0, i1), float64."""
    q0, q1 = i0 // 4, (i1 + 3) // 4
    ks = np.arange(k0, k1, dtype=np.uint64)[:, None]
    qs = np.arange(q0, q1, dtype=np.uint64)[None, :]
    w0, w1, w2, w3 = philox4x32_10(qs, ks, np.uint64(prob), np.uint64(0),
                                   seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    za, zb = box_muller(uniform_from_word(w0), uniform_from_word(w1))
    zc, zd = box_muller(uniform_from_word(w2), uniform_from_word(w3))
    out = np.empty((k1 - k0, 4 * (q1 - q0)))
    out[:, 0::4], out[:, 1::4], out[:, 2::4], out[:, 3::4] = za, zb, zc, zd
    off = i0 - 4 * q0
    return out[:, off:off + (i1 - i0)]


def uniform16_block(seed: int, prob: int, k0: int, k1: int, i0: int, i1: int) -> np.ndarray:
    """16-bit uniforms U[k, i] (int64) of the narrow-format sketch entries."""
    q0, q1 = i0 // 8, (i1 + 7) // 8
    ks = np.arange(k0, k1, dtype=np.uint64)[:, None]
    qs = np.arange(q0, q1, dtype=np.uint64)[None, :]
    w = philox4x32_10(qs, ks, np.uint64(prob), np.uint64(2), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = np.empty((k1 - k0, 8 * (q1 - q0)), dtype=np.int64)
    for t in range(8):
        out[:, t::8] = (w[t // 2].astype(np.int64) >> (16 * (t % 2))) & 0xFFFF
    off = i0 - 8 * q0
    return out[:, off:off + (i1 - i0)]


def normal_quantiles16() -> np.ndarray:
    """z[U] = Phi^-1((U + 1/2) / 2^16) for U = 0 .. 65535 (binary64).

    The lower half is evaluated where Phi^-1 is accurate (p < 1/2) and the
    upper half taken from it by symmetry, z[65535 - U] = -z[U]."""
    lo = ndtri((np.arange(32768, dtype=np.float64) + 0.5) / 65536.0)
    return np.concatenate([lo, -lo[::-1]])
