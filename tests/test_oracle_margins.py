"""The oracle's decision-margin bookkeeping (CPU only).

Slack loosens the image tolerance only at pixels whose skip or stop decision
lies within the float32 margin of its threshold, by the colour that decision
can move; these tests build single-pixel sequences with known alphas.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle

X = np.zeros(1)
Y = np.zeros(1)


def seq(alphas, colors, lno=False):
    """Gaussians on one pixel at offsets d_k from it with conic I, so alpha_k = o_k exp(-d_k^2/2)."""
    k = len(alphas)
    u = np.zeros(k)
    v = np.zeros(k)
    conic = np.tile([1.0, 0.0, 1.0], (k, 1))
    o = np.asarray(alphas, np.float64)           # d = 0: alpha = o exactly
    opa = np.log(o) if lno else o
    col = np.tile(np.asarray(colors, np.float64)[:, None], (1, 3))
    return u, v, conic, opa, col


def test_no_flags_far_from_thresholds():
    u, v, c, o, col = seq([0.5, 0.3, 0.2], [0.4, 0.9, 0.1])
    r = oracle.blend_tile(np.arange(3), X, Y, u, v, c, o, col, margins=(1e-4, 0.0))
    assert not r.flagged[0] and r.slack[0] == 0.0
    expect = 0.4 * 0.5 + 0.9 * 0.3 * 0.5 + 0.1 * 0.2 * 0.5 * 0.7
    assert abs(r.color[0][0, 0] - expect) < 1e-15


def test_skip_within_margin_is_flagged_with_its_contribution():
    a = (1.0 / 255.0) * (1.0 + 5e-5)              # passes, but within 1e-4 of the threshold
    u, v, c, o, col = seq([0.5, a], [0.2, 1.5])
    r = oracle.blend_tile(np.arange(2), X, Y, u, v, c, o, col, margins=(1e-4, 0.0))
    assert r.flagged[0]
    T_hi = 1.0 - 0.5 * (1 - 1e-4)                  # upper bound of T after the first pair
    assert math.isclose(r.slack[0], a * (1 + 1e-4) * T_hi * 1.5, rel_tol=1e-9)
    # outside the margin nothing is flagged
    u, v, c, o, col = seq([0.5, (1.0 / 255.0) * 1.01], [0.2, 1.5])
    r = oracle.blend_tile(np.arange(2), X, Y, u, v, c, o, col, margins=(1e-4, 0.0))
    assert not r.flagged[0]


def test_stop_within_margin_is_flagged_with_remaining_colour():
    # T after the first two pairs is 0.02 * 0.01; a third pair of alpha 0.5 takes it to
    # 1e-4 * (1 + 1e-5): just above the stop threshold, within the margin
    a3 = 1.0 - 1e-4 * (1 + 1e-5) / (0.02 * 0.01)
    u, v, c, o, col = seq([0.98, 0.99, a3, 0.3], [0.5, 0.5, 0.8, 1.2])
    r = oracle.blend_tile(np.arange(4), X, Y, u, v, c, o, col, margins=(1e-4, 0.0))
    assert r.flagged[0]
    T_before = 0.02 * 0.01
    assert r.slack[0] >= T_before * 1.2 * 0.99
    # the same sequence with a clear stop is not flagged and stops at the third pair
    u, v, c, o, col = seq([0.98, 0.99, 0.9, 0.3], [0.5, 0.5, 0.8, 1.2])
    r = oracle.blend_tile(np.arange(4), X, Y, u, v, c, o, col, margins=(1e-4, 0.0))
    assert not r.flagged[0] and r.n_proc[0][0] == 3


def test_exact_and_bit_level_stops_that_differ_give_mode_slack():
    # bit-level exp underestimates alpha by up to 3 %, so T can stay above 1e-4 where the
    # exact alpha takes it below
    P = [math.log(0.9), math.log(0.9), math.log(0.9), math.log(0.92), math.log(0.5)]
    u, v, c, o, col = seq(np.exp(P), [0.3, 0.4, 0.5, 0.6, 0.9], lno=True)
    r = oracle.blend_tile(np.arange(5), X, Y, u, v, c, o, col, modes=("fast-def", "fast-exact"),
                          margins=(2e-3, 2e-3))
    stops = [int(r.n_proc[m][0]) for m in range(2)]
    T_def = float(r.T[0][0])
    if stops[0] != stops[1]:
        assert r.mode_slack[0] > 0
    else:
        assert r.mode_slack[0] == 0
    assert 0.0 <= T_def <= 1.0


def test_fast_skip_margin_on_P():
    P = [math.log(0.6), -math.log(255.0) + 1e-3]     # second pair within 2e-3 of the threshold
    u, v, c, o, col = seq(np.exp(P), [0.3, 2.0], lno=True)
    r = oracle.blend_tile(np.arange(2), X, Y, u, v, c, o, col, modes=("fast-def",), margins=(2e-3, 2e-3))
    assert r.flagged[0] and r.slack[0] > 0


def test_per_pair_margin_scales_with_the_terms():
    """With (d_alpha, d_P, kappa, t_round), a pair's margin on P is d_P + kappa M, M the
    magnitude sum of its exponent's terms in tile-centre coordinates.  The pixel at (0, 0)
    sits at (-7.5, -7.5) from its tile's centre; a Gaussian on it with conic I has
    M = (15^2 + 15^2) / 2 + |ln o| = 225 + |ln o|."""
    kappa = 4e-6
    for off, flagged in ((5e-4, True), (2e-3, False), (-5e-4, True), (-2e-3, False)):
        P = [math.log(0.6), -math.log(255.0) + off]
        u, v, c, o, col = seq(np.exp(P), [0.3, 2.0], lno=True)
        M = 225.0 + abs(P[1])
        assert kappa * M > 5e-4 and kappa * M < 2e-3
        r = oracle.blend_tile(np.arange(2), X, Y, u, v, c, o, col, modes=("fast-def",),
                              margins=(1e-5, 0.0, kappa, 0.0))
        assert bool(r.flagged[0]) == flagged, (off, r.flagged[0])
        # with kappa = 0 only the absolute margin counts: nothing is within 1e-6
        r = oracle.blend_tile(np.arange(2), X, Y, u, v, c, o, col, modes=("fast-def",),
                              margins=(1e-5, 1e-6, 0.0, 0.0))
        assert not r.flagged[0]


def test_per_pair_margin_grows_with_distance_from_the_tile_centre():
    """The same pair evaluated at a pixel next to its tile's centre has smaller terms, so a
    P that is flagged at the tile corner is not flagged there."""
    P = [math.log(0.6), -math.log(255.0) + 5e-4]
    u, v, c, o, col = seq(np.exp(P), [0.3, 2.0], lno=True)
    Xc, Yc = np.full(1, 8.0), np.full(1, 8.0)         # 0.5 px from the centre (7.5, 7.5)
    uc, vc = u + 8.0, v + 8.0                          # the Gaussians on that pixel
    r = oracle.blend_tile(np.arange(2), Xc, Yc, uc, vc, c, o, col, modes=("fast-def",),
                          margins=(1e-5, 0.0, 4e-6, 0.0))
    # M = (1^2 + 1^2) / 2 + 5.54: kappa M = 2.6e-5 < 5e-4
    assert not r.flagged[0]


def test_transmittance_rounding_widens_the_stop_interval():
    """A pixel whose T ends a hair above the stop threshold is flagged once each blended pair
    may round T by one float32 unit, and not without that term."""
    alphas = [0.9] * 3 + [0.5]
    T = 0.1 ** 3 * 0.5                                  # 5e-4 after four pairs
    a5 = 1.0 - 1e-4 * (1.0 + 5e-7) / T                  # takes T to 1e-4 (1 + 5e-7)
    u, v, c, o, col = seq(alphas + [a5, 0.2], [0.5] * 6)
    r = oracle.blend_tile(np.arange(6), X, Y, u, v, c, o, col, margins=(0.0, 0.0, 0.0, 0.0))
    assert not r.flagged[0]
    r = oracle.blend_tile(np.arange(6), X, Y, u, v, c, o, col, margins=(0.0, 0.0, 0.0, 2.0 ** -22))
    assert r.flagged[0] and r.slack[0] > 0


def _fma32(a, b, c):
    """float32 fused multiply-add: the product of two float32 values is exact in float64."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


@pytest.mark.parametrize("log2", [False, True])
def test_float32_folded_exponent_stays_within_the_per_pair_margin(log2):
    """The per-pair margin kappa M on P must cover a float32 evaluation of the folded
    exponent.  This is a float32 replica of that evaluation, in the order the fast
    rasterizer takes it (Eqs. expand, c0, coeff, dot in tile-centre coordinates, then
    Eq. dual_pixel's step to the next row), over random conics (A, C up to 1/0.3, the
    dilated minimum), ln o down to -ln 255, means up to 60 px from the tile centre and
    every pixel offset of a tile.  Its error against float64 stays below kappa M / 8.
    With ``log2`` the coefficients are scaled by log2 e after folding (the hardware-exp2
    variants, the plain path's training variant among them), and P log2 e is compared."""
    rng = np.random.default_rng(7)
    f = np.float32
    n = 400_000
    A = rng.uniform(1e-3, 1 / 0.3, n)
    C = rng.uniform(1e-3, 1 / 0.3, n)
    B = rng.uniform(-0.999, 0.999, n) * np.sqrt(A * C)
    lno = np.log(rng.uniform(1 / 255, 1.0, n))
    u = rng.uniform(-60, 60, n) * rng.choice([0.05, 0.3, 1.0], n)
    v = rng.uniform(-60, 60, n) * rng.choice([0.05, 0.3, 1.0], n)
    x = rng.integers(0, 16, n) - 7.5
    y0 = 2.0 * rng.integers(0, 8, n) - 7.5          # the even row of a dual pixel
    second = rng.integers(0, 2, n).astype(bool)
    y = y0 + second
    dx, dy = x - u, y - v
    P64 = lno - 0.5 * (A * dx * dx + 2 * B * dx * dy + C * dy * dy)
    ax, ay = np.abs(x) + np.abs(u), np.abs(y) + np.abs(v)
    M = 0.5 * (A * ax * ax + 2 * np.abs(B) * ax * ay + C * ay * ay) + np.abs(lno)

    A32, B32, C32, L32, u32, v32 = (a.astype(f) for a in (A, B, C, lno, u, v))
    C0 = _fma32(A32 * u32, u32, _fma32(f(2) * B32 * u32, v32, C32 * v32 * v32))
    C1, C2, C3 = f(-0.5) * A32, -B32, f(-0.5) * C32
    C4 = _fma32(A32, u32, B32 * v32)
    C5 = _fma32(C32, v32, B32 * u32)
    C6 = _fma32(np.full(n, -0.5, f), C0, L32)
    if log2:
        l2e = f(1.4426950408889634)
        C1, C2, C3, C4, C5, C6 = (c * l2e for c in (C1, C2, C3, C4, C5, C6))
        P64 = P64 * (1.0 / math.log(2.0))
        M = M * (1.0 / math.log(2.0))
    x32, y32 = x.astype(f), y0.astype(f)
    x2, xy, y2 = x32 * x32, x32 * y32, y32 * y32
    y21 = _fma32(np.full(n, 2, f), y32, np.ones(n, f))
    P0 = _fma32(C1, x2, _fma32(C2, xy, _fma32(C3, y2, _fma32(C4, x32, _fma32(C5, y32, C6)))))
    P1 = P0 + _fma32(C2, x32, _fma32(C3, y21, C5))
    P32 = np.where(second, P1, P0).astype(np.float64)
    ratio = np.abs(P32 - P64) / M
    kappa = 4e-6                                     # the fast path's per-pair margin scale
    assert ratio.max() < kappa / 8, ratio.max()          # measured 3.6e-7, 4.0e-7 with log2
    # and the margin is not vacuous: the error is a sizeable multiple of one rounding of M
    assert ratio.max() > 2.0 ** -24


def test_plain_definition_with_tile_centre_margins():
    """The plain path's training variant evaluates the plain definition in the folded
    form: margin_frame="tile-centre" takes M in tile-centre coordinates for the plain
    mode too (with |ln o| for its opacity term).  A pair just above 1/255 at the tile
    corner (M = 225 + |ln o|) is flagged that way and not with the pixel frame (M = 0 for
    a Gaussian on the pixel)."""
    a = (1.0 / 255.0) * (1.0 + 5e-4)
    u, v, c, o, col = seq([0.5, a], [0.3, 2.0])
    mg = (1e-5, 0.0, 4e-6, 0.0)
    r = oracle.blend_tile(np.arange(2), X, Y, u, v, c, o, col, margins=mg, margin_frame="tile-centre")
    assert r.flagged[0] and r.slack[0] > 0
    r = oracle.blend_tile(np.arange(2), X, Y, u, v, c, o, col, margins=mg)
    assert not r.flagged[0]
    with pytest.raises(ValueError):
        oracle.blend_tile(np.arange(2), X, Y, u, v, c, o, col, margins=mg, margin_frame="pixels")


def test_adjoint_per_pair_margin():
    """The adjoint's skip margin grows by kappa M per pair (tile-centre frame) when its
    margins carry a fourth value; the image-space sums are unchanged."""
    from oracle import backward as OB
    a = (1.0 / 255.0) * (1.0 + 5e-4)
    u, v, c, o, col = seq([0.5, a], [0.3, 2.0])
    dC = np.ones((3, 1))
    bg = (0.1, 0.2, 0.3)
    plain = OB.blend_tile_adjoint(np.arange(2), X, Y, u, v, c, o, col, bg, dC)
    folded = OB.blend_tile_adjoint(np.arange(2), X, Y, u, v, c, o, col, bg, dC,
                                   margins=OB.DECISION_MARGINS + (4e-6,))
    assert not plain.flagged[0]
    assert folded.flagged[0] and (0, 1, "skip") in folded.near
    assert np.array_equal(plain.grad, folded.grad)
