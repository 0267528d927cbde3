"""Entry-wise comparison of the GPU sketch with the oracle (test helper).

The tolerance of each sampled entry is TOL_FACTOR times the oracle's rounding
scale for it (``oracle.sketch.error_scale``): binary32 accumulation over the
library's K-split (its length from ``ls_sketch_split_rows``) and the e4m3
MFMA's dot-product window (S's entries are the same on both sides).  The
scale is a root-sum-square
of per-step rounding bounds; a factor of 3 covers the tails of the largest of
many entries (the largest measured ratio of error to scale is about 2.7).
"""

import numpy as np
import torch

from oracle import sketch as osketch

TOL_FACTOR = 3.0


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sketch_ratio(L, P, At, b, s, seed, fmt, terms, rows, cols=None, plan=0, Y=None):
    """max over the sampled entries of |Y_gpu - Y_oracle| / (TOL_FACTOR * scale),
    the GPU sketch Y (s x (n+1)) and the ratios themselves."""
    colscale = fmt in ("f16", "e4m3")
    if Y is None:
        Y = host(L.ls_sketch(At, b, s, seed=seed, u_s=fmt, terms=terms, plan=plan)).T
    split = L.sketch_split_rows(At, b, s, u_s=fmt, terms=terms, plan=plan)
    n = P.n
    acols = list(range(n)) if cols is None else [c for c in cols if c < n]
    sub = np.ascontiguousarray(P.At[acols])
    # columns are independent (exponents, splits and products act per column)
    ref = osketch.sketch_rows(sub, P.b, s, seed, rows, fmt=fmt, terms=terms, colscale=colscale)
    scale = osketch.error_scale(sub, P.b, s, seed, rows, fmt, terms, colscale, split)
    got = Y[np.ix_(rows, acols + [n])]
    ratio = np.abs(got - ref) / (TOL_FACTOR * scale)
    return float(ratio.max()), Y, ratio
