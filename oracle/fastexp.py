"""Range-aware bit-level fast exponential (Sec. IV-B, Eq. fma_exp).

After opacity culling every surviving Gaussian-pixel pair has its folded
exponent P = p + ln o in [-ln 255, 0] (Eq. fast_exp_range).  The fast
exponential builds the IEEE-754 single-precision bit pattern of exp(P)
directly, after Schraudolph: the integer I(P) = floor(P 2^23 log2(e) +
2^23 (127 - sigma)) is reinterpreted as a float.  The paper calibrates
sigma = 0.045677 and states a relative error of about 0.03 on that range.

Closed form of the error (our derivation; the paper's appendix is not in this
copy): write P log2(e) - sigma = k + f with integer k and f in [0, 1).  The
bit pattern holds exponent k + 127 and mantissa fraction f (up to the floor,
which is below one mantissa unit), so exp^(P) = 2^k (1 + f) while
exp(P) = 2^(k + f + sigma).  Hence exp^/exp - 1 = 2^-sigma (1 + f) 2^-f - 1,
whose range over f in [0,1) is [2^-sigma - 1, 2^-sigma max_f (1+f) 2^-f - 1],
the maximum at f = 1/ln 2 - 1.
"""
from __future__ import annotations

import math

import numpy as np

SIGMA = 0.045677
LOG2E = 1.0 / math.log(2.0)
MANT = float(1 << 23)


def fast_exp(P) -> np.ndarray:
    """exp^(P): the float32 whose bits are I(P), evaluated in float64 as defined."""
    P = np.asarray(P, np.float64)
    I = np.floor(P * MANT * LOG2E + MANT * (127.0 - SIGMA))
    return I.astype(np.int64).astype(np.uint32).view(np.float32)


def fast_exp_rel_error(P) -> np.ndarray:
    """exp^(P) / exp(P) - 1 in float64."""
    P = np.asarray(P, np.float64)
    return fast_exp(P).astype(np.float64) / np.exp(P) - 1.0


def rel_error_envelope(sigma: float = SIGMA) -> tuple[float, float]:
    """[min, max] of 2^-sigma (1 + f) 2^-f - 1 over f in [0, 1), in closed form."""
    lo = 2.0 ** (-sigma) - 1.0
    f_star = 1.0 / math.log(2.0) - 1.0
    hi = 2.0 ** (-sigma) * (1.0 + f_star) * 2.0 ** (-f_star) - 1.0
    return lo, hi


def eps_star(sigma: float = SIGMA) -> float:
    """Largest |relative error| of exp^ (attained at f = 0 for the paper's sigma)."""
    lo, hi = rel_error_envelope(sigma)
    return max(-lo, hi)
