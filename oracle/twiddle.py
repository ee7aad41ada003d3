"""Reference roots of unity w_P^e = exp(-2 pi i e / P), correctly rounded to
binary64 with mpmath's cospi/sinpi at 60 significant digits.  Test infrastructure only."""
from __future__ import annotations

import numpy as np


def twiddles_ref(P: int, idx=None):
    import mpmath
    mpmath.mp.dps = 60
    if idx is None:
        idx = range(P)
    out = np.empty((len(idx), 2), dtype=np.float64)
    for j, e in enumerate(idx):
        a = mpmath.mpf(-2 * int(e)) / P        # exact for P = 2^k; else to 60 digits
        out[j, 0] = float(mpmath.cospi(a))     # cos(pi a), exact zeros at multiples of 1/2
        out[j, 1] = float(mpmath.sinpi(a))
    return out
