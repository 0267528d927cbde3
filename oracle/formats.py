"""Narrow floating-point formats used by the sketch (oracle, test use only).

Section 3 lets the sketch run in a precision u_s, A being held in that
precision (Algorithm 1's input).  Section 3.2 describes a one-sided
column scaling for narrow-range formats: divide every column by its largest
magnitude and multiply by a positive constant, then use R S^-1 as the
preconditioner.  The constant is taken as a power of two, so that the
scaling is exact.

Rounding is round-to-nearest, ties to even, computed on the exact binary64
value.  Subnormals are kept.  OCP e4m3 ("fn": no infinities, max 448)
saturates at +-448.
"""

import numpy as np

# (mantissa bits after the point, minimum normal exponent, largest finite value)
FORMATS = {
    "bf16": (7, -126, float.fromhex("0x1.fep127")),
    "f16": (10, -14, 65504.0),
    "e4m3": (3, -6, 448.0),
    "f32": (23, -126, float(np.finfo(np.float32).max)),
}

UNIT_ROUNDOFF = {
    "f64": 2.0 ** -53, "f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8, "e4m3": 2.0 ** -4,
}


def round_to(x, fmt: str) -> np.ndarray:
    """Round binary64 values to the nearest ``fmt`` value (ties to even)."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "f64":
        return x.copy()
    if fmt == "f32":
        return x.astype(np.float32).astype(np.float64)
    t, emin, fmax = FORMATS[fmt]
    ax = np.abs(x)
    # exponent of the leading bit, clamped to the subnormal range
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    # log2 may be off by one next to powers of two: fix it exactly
    e = np.where(ax >= np.ldexp(1.0, (e + 1).astype(np.int64)), e + 1, e)
    e = np.where(ax < np.ldexp(1.0, e.astype(np.int64)), e - 1, e)
    e = np.maximum(e, emin)
    quantum = np.ldexp(1.0, (e - t).astype(np.int64))
    q = np.round(x / quantum) * quantum          # np.round: ties to even, exact here
    if fmt == "e4m3":
        q = np.clip(q, -fmax, fmax)
    else:
        q = np.where(np.abs(q) > fmax, np.copysign(np.inf, q), q)
    return q


def column_exponents(M: np.ndarray, fmt: str) -> np.ndarray:
    """Largest integer e_j with max_i |M_ij| * 2^e_j <= largest finite value of ``fmt``.

    Columns that are entirely zero get e_j = 0.  Formats whose range equals
    binary32's (bf16, f32) and f64 are not scaled (e_j = 0).
    """
    ncol = M.shape[1]
    if fmt not in ("f16", "e4m3"):
        return np.zeros(ncol, dtype=np.int32)
    fmax = FORMATS[fmt][2]
    mx = np.max(np.abs(M), axis=0)
    e = np.zeros(ncol, dtype=np.int32)
    for j in range(ncol):
        if mx[j] == 0.0:
            continue
        f, E = np.frexp(mx[j])          # mx = f * 2^E, f in [0.5, 1)
        F, G = np.frexp(fmax)
        ej = G - E if f <= F else G - E - 1
        assert mx[j] * 2.0 ** ej <= fmax < mx[j] * 2.0 ** (ej + 1)
        e[j] = ej
    return e


def split_terms(M: np.ndarray, fmt: str, terms: int) -> list:
    """Write M as a sum of ``terms`` arrays each exactly representable in ``fmt``.

    T_1 = fl(M), T_2 = fl(M - T_1), ...; the differences are exact in binary64.
    """
    out, rem = [], np.asarray(M, dtype=np.float64)
    for _ in range(terms):
        t = round_to(rem, fmt)
        out.append(t)
        rem = rem - t
    return out
