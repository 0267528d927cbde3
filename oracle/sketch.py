"""Algorithm 1, the sketch: Y = Omega [A b] (oracle, test use only).

Definition (Section 2 and Algorithm 1; the sketch of [A b] rather than of A
alone is the reading taken here of how Q^T Omega b in Algorithm 2's
sketch-and-solve start is obtained without forming Q):

    M   = [A b] * diag(2^e)                 (Section 3.2 column scaling; e = 0 for
                                             bf16, f32 and f64)
    M_q = T_1 + ... + T_terms,  T_t = fl_us(M - T_1 - ... - T_{t-1})
                                            (A held in the sketch's precision;
                                             terms > 1 is a multi-term split)
    S_q = fl_us(Phi^-1((U + 1/2) / 2^16))   (narrow formats: 16-bit uniforms U,
                                             ``philox.uniform16_block``; the f64
                                             sketch uses ``philox.gaussian_block``)
    Y   = (1/sqrt(s)) * (S_q M_q) * diag(2^-e)

computed here with exact binary64 operands and a binary64 matrix product.
"""

import numpy as np

from . import formats, philox


_QUANTILES = {}


def format_quantiles(fmt):
    """The 2^16 possible entries of S in a narrow format: fl_fmt(z[U])."""
    if fmt not in _QUANTILES:
        _QUANTILES[fmt] = formats.round_to(philox.normal_quantiles16(), fmt)
    return _QUANTILES[fmt]


def quantised_gaussian_block(seed, prob, k0, k1, i0, i1, fmt):
    """S entries as the sketch uses them (float64 array): binary64 Box-Muller
    values for the f64 sketch, rounded 16-bit quantiles for a narrow format."""
    if fmt == "f64":
        return philox.gaussian_block(seed, prob, k0, k1, i0, i1)
    return format_quantiles(fmt)[philox.uniform16_block(seed, prob, k0, k1, i0, i1)]


def scaled_operand(At: np.ndarray, b: np.ndarray, fmt: str, terms: int, colscale: bool):
    """(M_q, e): the quantised, column-scaled [A b] (m x (n+1)) and the exponents."""
    m, n = At.shape[1], At.shape[0]
    M = np.empty((m, n + 1))
    M[:, :n] = At.T
    M[:, n] = b
    e = formats.column_exponents(M, fmt) if colscale else np.zeros(n + 1, dtype=np.int32)
    Ms = M * np.ldexp(1.0, e.astype(np.int64))[None, :]
    if fmt == "f64":
        return Ms, e
    Mq = np.sum(formats.split_terms(Ms, fmt, terms), axis=0)
    return Mq, e


def sketch(At: np.ndarray, b: np.ndarray, s: int, seed: int, prob: int = 0, fmt: str = "f64",
           terms: int = 1, colscale: bool = False, chunk: int = 4096):
    """Y = Omega [A b] as defined in the module docstring.

    Returns (Y (s x (n+1)) float64, e (n+1) int32).
    """
    Mq, e = scaled_operand(At, b, fmt, terms, colscale)
    m = Mq.shape[0]
    Y = np.zeros((s, Mq.shape[1]))
    for i0 in range(0, m, chunk):
        i1 = min(m, i0 + chunk)
        S = quantised_gaussian_block(seed, prob, 0, s, i0, i1, fmt)
        Y += S @ Mq[i0:i1]
    Y *= 1.0 / np.sqrt(s)
    Y *= np.ldexp(1.0, -e.astype(np.int64))[None, :]
    return Y, e


def sketch_rows(At, b, s, seed, rows, prob=0, fmt="f64", terms=1, colscale=False, chunk=65536):
    """Selected rows Y[rows, :] of the same sketch (each costs m (n+1) flops)."""
    Mq, e = scaled_operand(At, b, fmt, terms, colscale)
    m = Mq.shape[0]
    out = np.zeros((len(rows), Mq.shape[1]))
    for t, k in enumerate(rows):
        acc = np.zeros(Mq.shape[1])
        for i0 in range(0, m, chunk):
            i1 = min(m, i0 + chunk)
            S = quantised_gaussian_block(seed, prob, k, k + 1, i0, i1, fmt)
            acc += S[0] @ Mq[i0:i1]
        out[t] = acc
    out *= 1.0 / np.sqrt(s)
    out *= np.ldexp(1.0, -e.astype(np.int64))[None, :]
    return out


# ------------------------------------------------------------------ rounding-error scale
# Relative precision, with respect to the largest of its products, of one
# 32-term dot product of an MFMA (measured on gfx950 for random operands):
# e4m3 products are aligned to the largest one within a window of about 17
# bits, so that each of the 32 may lose up to 2^-17 of the largest, about
# sqrt(32) 2^-17 = 2^-14.5 in all (2^-17.6 per step for products of few bits,
# about 2^-14.7 for random operands); bf16 and fp16 products to about 2^-20.8
# of the largest (2^-20 allowed), rather than one binary32 rounding.  The
# longer e4m3 products of the f8f6f4 forms are counted as consecutive 32-term
# steps: a 128-term one (16x16x128) showed the same errors as four of them,
# and the 64-term one (32x32x64) stays within that model in the parity tests.
DOT_PRECISION = {"e4m3": 2.0 ** -14, "bf16": 2.0 ** -20, "f16": 2.0 ** -20}


def error_scale(At, b, s, seed, rows, fmt, terms, colscale, split_rows, prob=0, kstep=32):
    """Scale of the rounding error of selected rows of the narrow-format sketch
    computed with binary32 accumulation (test use).

    Section 3.1 bounds the sketch's error by a casting term and the matrix
    product's accumulation term.  With the cast operands (S_q, M_q) fixed, an
    evaluation that sums the products of each ``split_rows``-row split in
    binary32, one rounding per ``kstep`` rows, and adds the split sums in
    binary64 deviates from the exact product by rounding errors of at most
    u32 |P_t| at each step t, P_t the running sum after step t.  Modelled as
    independent, they add up to about

        sigma_acc[k, j] = u32 * sqrt(sum_t P_t[k, j]^2),

    where each step's dot product of ``kstep`` products may itself carry an
    error of d |p|_max (d = DOT_PRECISION[fmt], |p|_max the largest of its
    products, per part T_t of the split):

        sigma_dot[k, j] = d * sqrt(sum_t sum_steps |p|_max^2),

    (S_q itself is exact on both sides: its entries are table values.)

    Returns (sigma_acc + sigma_dot) / sqrt(s) * 2^-e_j for the sampled rows and
    every column of [At^T b] (len(rows) x (n+1))."""
    Mq, e = scaled_operand(At, b, fmt, terms, colscale)
    m, nc = Mq.shape
    d = DOT_PRECISION[fmt]
    if d:
        n = At.shape[0]
        M = np.empty((m, n + 1))
        M[:, :n] = At.T
        M[:, n] = b
        parts = formats.split_terms(M * np.ldexp(1.0, e.astype(np.int64))[None, :], fmt, terms)
    out = np.empty((len(rows), nc))
    L = int(split_rows) if split_rows else m
    for r, k in enumerate(rows):
        Sq = quantised_gaussian_block(seed, prob, k, k + 1, 0, m, fmt)[0]
        acc2 = np.zeros(nc)
        for c0 in range(0, m, L):
            c1 = min(m, c0 + L)
            prod = Sq[c0:c1, None] * Mq[c0:c1]
            nblk = -(-(c1 - c0) // kstep)
            pad = np.zeros((nblk * kstep, nc))
            pad[:c1 - c0] = prod
            P = np.cumsum(pad.reshape(nblk, kstep, nc).sum(axis=1), axis=0)
            acc2 += np.sum(P * P, axis=0)
        sig_acc = 2.0 ** -24 * np.sqrt(acc2)
        sig_dot = np.zeros(nc)
        if d:
            nblk = -(-m // kstep)
            for T in parts:
                pad = np.zeros((nblk * kstep, nc))
                pad[:m] = np.abs(Sq[:, None] * T)
                sig_dot += np.sum(pad.reshape(nblk, kstep, nc).max(axis=1) ** 2, axis=0)
            sig_dot = d * np.sqrt(sig_dot)
        out[r] = (sig_acc + sig_dot) / np.sqrt(s) * np.ldexp(1.0, -e.astype(np.int64))
    return out


# ------------------------------------------------------------------ sparse sign embedding
SPARSE_MAX_WORDS = 256   # Philox words a column may use before the draw is declared failed


def sparse_sign_pattern(seed: int, prob: int, m: int, s: int, zeta: int):
    """Nonzeros of the sparse sign embedding of Section 2.

    Column i of Omega (the column that multiplies row i of [A b]) has zeta
    nonzeros at distinct rows chosen uniformly at random, each +1 or -1 with
    probability 1/2, scaled by 1/sqrt(zeta) (the reading taken here of the
    printed scale; it makes E[Omega^T Omega] = I as the embedding definition of
    Section 2 requires).  The random choices are read from the words of the
    Philox4x32-10 blocks with counter (i, t, prob, 1), t = 0, 1, ..., key
    (seed mod 2^32, seed / 2^32), in order: word w proposes row
    floor(w s / 2^32), negative when w is odd; a proposal equal to an earlier
    row of the same column is skipped.

    Returns (H, S): (m, zeta) int64 rows and (m, zeta) float64 signs, in
    the order drawn.
    """
    if not (2 <= zeta <= s):
        raise ValueError("need 2 <= zeta <= s")
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    rows = np.arange(m, dtype=np.uint64)
    H = np.full((m, zeta), -1, dtype=np.int64)
    S = np.zeros((m, zeta))
    count = np.zeros(m, dtype=np.int64)
    t = 0
    while np.any(count < zeta):
        if 4 * t >= SPARSE_MAX_WORDS:
            raise RuntimeError("sparse sign draw did not finish")
        words = philox.philox4x32_10(rows, np.uint64(t), np.uint64(prob), np.uint64(1), k0, k1)
        for w in words:
            w64 = w.astype(np.uint64)
            h = ((w64 * np.uint64(s)) >> np.uint64(32)).astype(np.int64)
            sign = np.where((w64 & np.uint64(1)) == 1, -1.0, 1.0)
            dup = np.any(H == h[:, None], axis=1)
            take = (count < zeta) & ~dup
            idx = np.nonzero(take)[0]
            H[idx, count[idx]] = h[idx]
            S[idx, count[idx]] = sign[idx]
            count[idx] += 1
        t += 1
    return H, S


def sparse_sketch(At: np.ndarray, b: np.ndarray, s: int, seed: int, zeta: int, prob: int = 0,
                  chunk: int = 2048):
    """Y = Omega [A b] for the sparse sign embedding (Section 2), binary64.

    Every row i of [A b] is added, with its signs, into the zeta rows of Y
    that column i of Omega selects, rows i in increasing order; Y is then
    multiplied by 1/sqrt(zeta).
    """
    m, n = At.shape[1], At.shape[0]
    H, S = sparse_sign_pattern(seed, prob, m, s, zeta)
    Y = np.zeros((s, n + 1))
    for i0 in range(0, m, chunk):
        i1 = min(m, i0 + chunk)
        M = np.empty((i1 - i0, n + 1))
        M[:, :n] = At[:, i0:i1].T
        M[:, n] = b[i0:i1]
        contrib = S[i0:i1, :, None] * M[:, None, :]          # (rows, zeta, n+1), exact
        np.add.at(Y, H[i0:i1].ravel(), contrib.reshape(-1, n + 1))
    Y *= 1.0 / np.sqrt(float(zeta))
    return Y


def sparse_sketch_rows(At: np.ndarray, b: np.ndarray, s: int, seed: int, zeta: int, rows, prob: int = 0):
    """Selected rows of the sparse sign sketch, with the additions of
    ``sparse_sketch`` in the same order (its sources in increasing row i)."""
    m, n = At.shape[1], At.shape[0]
    H, S = sparse_sign_pattern(seed, prob, m, s, zeta)
    out = np.zeros((len(rows), n + 1))
    for t, r in enumerate(rows):
        src, k = np.nonzero(H == r)          # row-major order: increasing i
        acc = np.zeros(n + 1)
        for i, kk in zip(src, k):
            row = np.empty(n + 1)
            row[:n] = At[:, i]
            row[n] = b[i]
            acc += S[i, kk] * row
        out[t] = acc
    out *= 1.0 / np.sqrt(float(zeta))
    return out
