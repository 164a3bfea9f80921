"""Front-to-back alpha blending of one tile (Sec. III-D, Sec. IV-B).

For a pixel at x and a Gaussian with projected mean (u, v), conic (A, B, C)
and opacity o, Eq. power gives the exponent
    p = -1/2 (A dx^2 + 2 B dx dy + C dy^2),   (dx, dy) = (x - u, y - v),
Eq. alpha_computation / opacity_clamped give alpha = min(0.99, o exp(p)),
and the Gaussians of the tile are composited front to back:
    C += alpha T c,   T <- T (1 - alpha).
The fast path folds ln o into the exponent (Eq. folded_exponent,
P = p + ln o) and takes alpha = min(0.99, exp(P)), or with the bit-level
exponential of Eq. fma_exp, alpha = min(0.99, exp^(P)).

Readings of what the paper leaves to 3DGS:
* a pair is skipped when alpha < 1/255; in the fast path the test is made on
  P < -ln 255, which is the same test in exact arithmetic and keeps exactly the
  pairs whose P lies in [-ln 255, 0] (Eq. fast_exp_range).  Testing exp^(P)
  instead would drop pairs the exact path keeps, since exp^(-ln 255) < 1/255;
* blending of a pixel stops at the first pair whose T (1 - alpha) would fall
  below 1e-4; that pair is not blended;
* the output is C + T bg.

``blend_tile`` evaluates one or more alpha definitions in lockstep over the
same sorted list.  The first is the primary result.  Two pieces of test
bookkeeping run beside it, and neither changes the primary result:
* ``margins`` (relative uncertainty of alpha, absolute uncertainty of P)
  describes how far a float32 implementation of the primary definition may
  stray; pairs whose skip or stop decision lies within that margin are
  flagged, and the colour that the decision puts at stake is accumulated as a
  per-pixel slack (alpha T c_max for a skip, T c_max for a stop, after which
  tracking of that pixel ends);
* when the definitions stop a pixel at different pairs, the larger T at the
  first difference times c_max is recorded as ``mode_slack``.

The margins may also scale with each pair.  A float32 evaluation of the
exponent rounds every term it adds, so its error is bounded by a multiple of
the sum of the terms' magnitudes, not of the result.  With ``margins`` =
(delta_alpha_rel, delta_P_abs, kappa, t_round), each pair's margins on P and on
the relative alpha grow by kappa M, where M bounds the magnitudes of the terms
of its exponent in the frame the fast rasterizer folds them in (coordinates
relative to the centre of the pixel's 16x16 tile, Sec. IV-B):
    M = 1/2 (|A| (|x| + |u|)^2 + 2 |B| (|x| + |u|) (|y| + |v|) + |C| (|y| + |v|)^2) + |ln o|
(for the plain mode, with the pixel-to-mean offsets of Eq. power:
M = 1/2 (|A| dx^2 + 2 |B| |dx dy| + |C| dy^2)), and every blended pair widens
the transmittance interval by the relative rounding t_round of one float32
update.
c_max is the largest colour component of any pair at the pixel that passes,
or may pass, the skip test.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .fastexp import fast_exp
from .project import LN255

ALPHA_MAX = 0.99
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4

MODES = ("plain", "fast-exact", "fast-def")


@dataclass
class BlendResult:
    color: list          # per mode: [3, npix] float64 (C + T bg)
    T: list              # per mode: [npix] final transmittance
    n_proc: list         # per mode: [npix] pairs visited (the stopping pair included)
    n_blend: list        # per mode: [npix] pairs blended (past the skip test, not the stopping one)
    c_max: np.ndarray    # [npix]
    slack: np.ndarray    # [npix] decision slack of the primary mode (colour units)
    flagged: np.ndarray  # [npix] bool, a decision of the primary mode was within margin
    mode_slack: np.ndarray  # [npix] slack from differing stop decisions between modes


def _alpha(mode: str, p: np.ndarray, opa: float):
    """(clamped alpha, unclamped alpha, skip mask, P) of one Gaussian for all pixels."""
    if mode == "plain":
        raw = opa * np.exp(p)
        return np.minimum(ALPHA_MAX, raw), raw, raw < ALPHA_MIN, None
    P = p + opa
    if mode == "fast-exact":
        raw = np.exp(P)
    else:
        # far below the skip threshold the bit pattern would leave the float range;
        # those pairs are skipped, so their value is irrelevant
        raw = fast_exp(np.maximum(P, -80.0)).astype(np.float64)
    return np.minimum(ALPHA_MAX, raw), raw, P < -LN255, P


def blend_tile(gauss_ids, X, Y, u, v, conic, opa, color, modes=("plain",), bg=(0.0, 0.0, 0.0),
               margins=None, margin_frame=None) -> BlendResult:
    """Blend the sorted Gaussians ``gauss_ids`` at pixel positions X, Y (float arrays).

    ``opa`` holds opacity o for the plain mode and ln o for the fast modes.
    ``margins`` = (delta_alpha_rel, delta_P_abs[, kappa, t_round]) turns on
    decision tracking.  ``margin_frame`` names the coordinates the per-pair
    magnitude M is taken in: "pixel" (offsets from the pixel, Eq. power as
    written) or "tile-centre" (the folded form); by default the plain mode's
    is "pixel" and the fast modes' "tile-centre".  It changes no result, only
    which decisions are flagged.
    """
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    n = X.size
    k = len(modes)
    T = [np.ones(n) for _ in range(k)]
    C = [np.zeros((3, n)) for _ in range(k)]
    done = [np.zeros(n, bool) for _ in range(k)]
    n_proc = [np.zeros(n, np.int64) for _ in range(k)]
    n_blend = [np.zeros(n, np.int64) for _ in range(k)]
    c_max = np.zeros(n)
    slack_units = np.zeros(n)
    flagged = np.zeros(n, bool)
    tracking = np.ones(n, bool)
    T_lo = np.ones(n)
    T_hi = np.ones(n)
    mode_slack_T = np.zeros(n)
    modes_agree = np.ones(n, bool)
    mg = tuple(margins) if margins is not None else (0.0, 0.0)
    d_alpha0, d_P0 = mg[0], mg[1]
    kappa = mg[2] if len(mg) > 2 else 0.0
    t_round = mg[3] if len(mg) > 3 else 0.0
    frame = margin_frame or ("pixel" if modes[0] == "plain" else "tile-centre")
    if frame not in ("pixel", "tile-centre"):
        raise ValueError(margin_frame)
    # pixel coordinates relative to the centre of their 16x16 tile
    tcx = np.floor(X / 16.0) * 16.0 + 7.5
    tcy = np.floor(Y / 16.0) * 16.0 + 7.5

    for g in gauss_ids:
        if all(dm.all() for dm in done):
            break
        dx = X - u[g]
        dy = Y - v[g]
        A, B, Cc = conic[g]
        p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        if kappa > 0.0:
            if frame == "pixel":
                M = 0.5 * (abs(A) * dx * dx + 2.0 * abs(B) * np.abs(dx * dy) + abs(Cc) * dy * dy)
            else:
                ax = np.abs(X - tcx) + np.abs(u[g] - tcx)
                ay = np.abs(Y - tcy) + np.abs(v[g] - tcy)
                lno = opa[g] if modes[0] != "plain" else (np.log(opa[g]) if opa[g] > 0.0 else 0.0)
                M = 0.5 * (abs(A) * ax * ax + 2.0 * abs(B) * ax * ay + abs(Cc) * ay * ay) + abs(lno)
            d_alpha = d_alpha0 + kappa * M
            d_P = d_P0 + kappa * M
        else:
            d_alpha, d_P = d_alpha0, d_P0
        col = color[g]
        T_before = [t.copy() for t in T]
        any_active = ~np.logical_and.reduce(done)
        for m, mode in enumerate(modes):
            a, raw, skip, P = _alpha(mode, p, opa[g])
            active = ~done[m]
            n_proc[m] += active
            blend = active & ~skip
            Tn = T[m] * (1.0 - a)
            stop = blend & (Tn < T_MIN)
            done[m] |= stop
            blend &= ~stop
            n_blend[m] += blend
            C[m] += np.where(blend, a * T[m], 0.0)[None, :] * col[:, None]
            T[m] = np.where(blend, Tn, T[m])
            if m == 0:
                if mode == "plain":
                    maybe_pass = raw * (1.0 + d_alpha) >= ALPHA_MIN
                    amb_skip = maybe_pass & (raw * (1.0 - d_alpha) < ALPHA_MIN)
                else:
                    maybe_pass = P >= -LN255 - d_P
                    amb_skip = maybe_pass & (P < -LN255 + d_P)
                c_max = np.where(any_active & maybe_pass, np.maximum(c_max, col.max()), c_max)
                if margins is not None:
                    live = tracking & active
                    a_lo = np.minimum(ALPHA_MAX, raw * (1.0 - d_alpha))
                    a_hi = np.minimum(ALPHA_MAX, raw * (1.0 + d_alpha))
                    passes = live & ~skip & ~amb_skip
                    amb = live & amb_skip
                    slack_units += np.where(amb, a_hi * T_hi, 0.0)
                    flagged |= amb
                    new_lo = np.where(passes | amb, T_lo * (1.0 - a_hi) * (1.0 - t_round), T_lo)
                    new_hi = np.where(passes, T_hi * (1.0 - a_lo) * (1.0 + t_round), T_hi)
                    amb_stop = (passes | amb) & (new_lo < T_MIN) & (new_hi >= T_MIN)
                    slack_units += np.where(amb_stop, T_hi, 0.0)
                    flagged |= amb_stop
                    tracking &= ~amb_stop
                    T_lo = np.where(tracking, new_lo, T_lo)
                    T_hi = np.where(tracking, new_hi, T_hi)
        if k > 1:
            differ = np.zeros(n, bool)
            for m in range(1, k):
                differ |= done[m] != done[0]
            first = modes_agree & differ
            if first.any():
                worst = np.max(np.stack(T_before), axis=0)
                mode_slack_T = np.where(first, worst, mode_slack_T)
                modes_agree &= ~differ

    bg = np.asarray(bg, np.float64)
    colors = [C[m] + T[m][None, :] * bg[:, None] for m in range(k)]
    return BlendResult(color=colors, T=T, n_proc=n_proc, n_blend=n_blend, c_max=c_max,
                       slack=slack_units * c_max, flagged=flagged,
                       mode_slack=mode_slack_T * c_max)
