"""The FP64 oracle against the paper's printed values, closed forms, library
routines, brute force and invariants (CPU only)."""
from __future__ import annotations

import importlib
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import workloads as wl
from oracle_checks import (brute_force_image, check_brute_force, check_depth_order_and_stop,
                           check_fast_exp_envelope, check_off_axis_jacobian, check_rotation,
                           check_sh_basis, check_single_gaussian, fp16_round_exact)

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
TILES = importlib.import_module("oracle.tiles")
FASTEXP = importlib.import_module("oracle.fastexp")


# ---- Sec. IV-A key encoding -------------------------------------------------------------

def test_key_split_worked_example():
    g = GOLDEN["key_split_example"]
    p = oracle.frame_plan(g["width"], g["height"])
    assert (p.tiles_x, p.tiles_y, p.n_tiles) == (g["tiles_x"], g["tiles_y"], g["n_tiles"])
    assert (p.b_t, p.b_d) == (g["b_t"], g["b_d"])
    assert p.depth_levels == g["depth_levels"]


def test_key_split_edges():
    assert oracle.key_bits(1) == (1, 31)          # reading: at least one tile bit
    assert oracle.key_bits(2) == (1, 31)
    assert oracle.key_bits(3) == (2, 30)
    assert oracle.key_bits(256) == (8, 24)
    assert oracle.key_bits(257) == (9, 23)
    for n in range(1, 5000):
        bt, bd = oracle.key_bits(n)
        assert (1 << bt) >= n and (bt == 1 or (1 << (bt - 1)) < n) and bt + bd == 32


def test_sort_budgets_from_paper():
    g = GOLDEN["sort"]
    assert g["baseline_key_bits"] // 8 == g["baseline_passes"]
    assert g["fast_key_bits"] // 8 == g["fast_passes"]
    assert g["baseline_entry_bytes"] == 8 + 4


@settings(max_examples=200, deadline=None)
@given(st.floats(0.2, 100.0), st.floats(0.2, 100.0), st.integers(12, 31))
def test_depth_quantiser_monotone(d1, d2, b_d):
    zn, zf = 0.2, 100.0
    q = TILES.quantize_depth(np.array([d1, d2]), zn, zf, b_d)
    if d1 <= d2:
        assert q[0] <= q[1]
    step = (zf - zn) / ((1 << b_d) - 1)
    if abs(d1 - d2) >= step * (1 + 1e-9):
        assert q[0] != q[1]
    assert 0 <= q.min() and q.max() <= (1 << b_d) - 1


def test_depth_quantiser_bounds():
    q = TILES.quantize_depth(np.array([1.0, 2.0, 3.0]), 1.0, 3.0, 19)
    assert list(q) == [0, ((1 << 19) - 1) // 2, (1 << 19) - 1]


# ---- projection and colour ------------------------------------------------------------

def test_rotation_matches_scipy():
    assert check_rotation() < 1e-14


def test_sh_basis_matches_scipy():
    assert check_sh_basis() < 1e-12


def test_off_axis_jacobian_closed_form():
    assert check_off_axis_jacobian() < 1e-12


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_single_isotropic_gaussian_closed_form(path):
    assert check_single_gaussian(path=path) < 1e-12


def test_single_anisotropic_gaussian_closed_form():
    th = 0.7
    q = (math.cos(th / 2), 0.0, 0.0, math.sin(th / 2))        # rotation about the view axis
    assert check_single_gaussian(quat=q, scales=(0.09, 0.03, 0.05)) < 1e-12
    q = (0.8, 0.3, -0.4, 0.33)                                 # general rotation
    assert check_single_gaussian(quat=q, scales=(0.09, 0.03, 0.05)) < 1e-12


def test_depth_order_and_stop_closed_form():
    assert check_depth_order_and_stop() < 1e-12


# ---- tiling, sorting, ranges --------------------------------------------------------------

@pytest.mark.parametrize("path", ["plain", "fast"])
@pytest.mark.parametrize("seed", [5, 11])
def test_tiled_equals_brute_force(path, seed):
    assert check_brute_force(path=path, seed=seed) < 1e-12


@pytest.mark.parametrize("key64,alpha_extent", [(True, True), (False, False), (True, False)])
def test_fast_ablations_equal_brute_force(key64, alpha_extent):
    """The fast path keyed on float32 depth, or with the 3-sigma extent, still
    equals per-pixel blending in (key, index) order over the same rectangles."""
    for seed in (5, 11):
        assert check_brute_force("fast", seed, key64=key64, alpha_extent=alpha_extent) < 1e-12


def test_alpha_extent_changes_entries_not_the_image():
    """Sec. IV-A's opacity cull and alpha-ellipse extent only drop pairs whose
    P is below -ln 255, which the skip test rejects: the image is the same bit
    for bit, with fewer entries."""
    sc = wl.make_scene(3000, 1.0, -3.0, 0.5, 17)
    cam = wl.config_camera("small", width=96, height=80)
    arr = oracle.prepare_fast(oracle.quantize_scene(sc))
    a = oracle.render(arr, cam, "fast")
    b = oracle.render(arr, cam, "fast", alpha_extent=False)
    assert b.keys.size > a.keys.size
    for m in a.modes:
        assert np.array_equal(a.images[m], b.images[m])
    assert np.array_equal(a.n_blend, b.n_blend)


def test_ablated_storage_reads_the_fp32_scene():
    sc = wl.make_scene(500, 1.0, -3.0, 0.5, 19)
    fs = oracle.quantize_scene(sc)
    full = oracle.prepare_fast_ablated(sc, fs, int8_sh=False, fp16_geometry=False)
    assert np.array_equal(full["sh"], sc.sh.astype(np.float64))
    assert np.array_equal(full["quats"], sc.quats.astype(np.float64))
    assert np.array_equal(full["means"], sc.means.astype(np.float64))
    lno = full["log_opacity"]
    # float32 rounding moves ln o by at most half an ulp, 2^-24 |ln o|, which is
    # the relative change of o
    assert np.all(np.abs(np.exp(lno) - sc.opacity) <= (2.0 ** -24 * np.abs(lno) + 1e-12) * 1.001 * sc.opacity)
    assert np.array_equal(lno, lno.astype(np.float32).astype(np.float64))
    only_sh = oracle.prepare_fast_ablated(sc, fs, int8_sh=False)
    dq = oracle.prepare_fast(fs)
    assert np.array_equal(only_sh["quats"], dq["quats"]) and np.array_equal(only_sh["sh"], full["sh"])


def test_empty_frame():
    sc = wl.make_scene(20, 1.0, -3.0, 0.3, 3)
    cam = wl.look_at_camera((0, 0, 30.0), (0, 0, 40.0), (0, 1, 0), 60.0, 40, 40, 1.0, 2.0)
    fr = oracle.render(oracle.prepare_plain(sc), cam, "plain")
    assert fr.keys.size == 0 and not fr.proj.visible.any()
    assert np.all(fr.ranges == 0) and np.all(fr.image == 0.0) and np.all(fr.T_final == 1.0)


def test_one_pixel_image():
    sc = wl.make_scene(200, 1.0, -1.5, 0.3, 4)
    cam = wl.look_at_camera((0, 0, -3.0), (0, 0, 0), (0, 1, 0), 60.0, 1, 1, 1.268, 4.732)
    fr = oracle.render(oracle.prepare_plain(sc), cam, "plain")
    assert fr.plan.n_tiles == 1 and fr.plan.b_t == 1
    assert fr.ranges[0, 1] == fr.keys.size
    ref = brute_force_image(oracle.prepare_plain(sc), cam, "plain", "plain")
    assert np.max(np.abs(fr.image - ref)) < 1e-12


def test_sorted_entries_grouped_and_stable():
    sc = wl.config_scene("small", n=3000)
    cam = wl.config_camera("small")
    for path, arr in (("plain", oracle.prepare_plain(sc)),
                      ("fast", oracle.prepare_fast(oracle.quantize_scene(sc)))):
        fr = oracle.render(arr, cam, path, blend=False)
        k, g = fr.sorted_keys, fr.sorted_gauss
        assert np.all(k[1:] >= k[:-1])
        ties = k[1:] == k[:-1]
        assert np.all(g[1:][ties] > g[:-1][ties])
        # every (Gaussian, tile) pair appears once and matches its rectangle
        shift = fr.key_shift
        tiles = (k >> np.uint64(shift)).astype(np.int64)
        rect = fr.proj.rect[g]
        tx, ty = tiles % fr.plan.tiles_x, tiles // fr.plan.tiles_x
        assert np.all((rect[:, 0] <= tx) & (tx <= rect[:, 1]) & (rect[:, 2] <= ty) & (ty <= rect[:, 3]))
        n_expect = np.sum((fr.proj.rect[:, 1] - fr.proj.rect[:, 0] + 1) *
                          (fr.proj.rect[:, 3] - fr.proj.rect[:, 2] + 1) * fr.proj.visible)
        assert k.size == n_expect
        assert len(set(zip(g.tolist(), tiles.tolist()))) == k.size
        for t in range(fr.plan.n_tiles):
            a, b = fr.ranges[t]
            assert np.all(tiles[a:b] == t)


# ---- compact storage (Eq. quant) ------------------------------------------------------------

def test_sh_quantiser_properties():
    rng = np.random.default_rng(0)
    sh = rng.normal(0, 0.3, size=(500, 16, 3)).astype(np.float32)
    sh[3] = 0.0                                  # all-zero Gaussian
    sh[4, 1:4, 2] = 0.0                          # zero degree-1 block in one channel
    q, s = oracle.quantize_sh(sh)
    deq = oracle.dequantize_scene(oracle.FastScene(
        means=np.zeros((500, 3), np.float32), quats=np.zeros((500, 4), np.float16),
        scales=np.zeros((500, 3), np.float16), log_opacity=np.zeros(500, np.float16),
        sh_q=q, sh_scale=s))["sh"]
    slices = [slice(0, 1), slice(1, 4), slice(4, 9), slice(9, 16)]
    for d, sl in enumerate(slices):
        sd = s[:, d, :].astype(np.float64)[:, None, :]
        err = np.abs(sh[:, sl, :].astype(np.float64) - deq[:, sl, :])
        assert np.all(err <= sd / 2 + 1e-300)
        amax = np.max(np.abs(q[:, sl, :].astype(np.int64)), axis=1)
        # with an FP16-normal scale the largest coefficient maps to +-127; a subnormal
        # scale is coarse and may round up far enough to leave it below
        normal = s[:, d, :].astype(np.float64) >= 2.0 ** -14
        assert np.all(amax[normal] == 127)
    assert np.all(q[3] == 0) and np.all(s[3] == 0)
    assert np.all(q[4, 1:4, 2] == 0) and s[4, 1, 2] == 0
    assert q.dtype == np.int8 and np.abs(q.astype(np.int64)).max() <= 127


def test_fp16_rounding_is_nearest_even():
    rng = np.random.default_rng(1)
    xs = list(np.exp(rng.uniform(-20, 11, 3000)) * rng.choice([-1, 1], 3000))
    # exact ties between neighbouring halves, normal and subnormal
    for k in range(200):
        e = int(rng.integers(-24, 15))
        m = int(rng.integers(0, 1024))
        ulp = 2.0 ** (max(e, -14) - 10)
        xs.append((2.0 ** max(e, -14) if e >= -14 else 0.0) + (m + 0.5) * ulp)
    for x in xs:
        assert float(np.float64(x).astype(np.float16)) == fp16_round_exact(float(x)), x


def test_byte_budgets():
    g = GOLDEN["byte_budgets"]
    assert 3 * 4 + 3 * 4 + 4 * 4 + 4 == g["plain_geometry"]
    assert 16 * 3 * 4 == g["plain_sh"]
    assert g["plain_geometry"] + g["plain_sh"] == g["plain_total"]
    ours = 3 * 4 + 4 * 2 + 3 * 2 + 2 + 48 + 12 * 2          # mean, quat, scale, ln o, SH, SH scales
    assert ours == 100
    assert abs(1 - g["compact_total_approx"] / g["plain_total"] - g["reduction_percent"] / 100) < 1e-3


# ---- the bit-level exponential (Eq. fma_exp) -----------------------------------------------------

def test_fast_exp_envelope_closed_form():
    assert FASTEXP.SIGMA == GOLDEN["fast_exp"]["sigma"]
    assert check_fast_exp_envelope() < 2e-6


def test_fast_exp_error_matches_paper():
    lo, hi = FASTEXP.rel_error_envelope()
    eps = FASTEXP.eps_star()
    assert round(eps, 2) == GOLDEN["fast_exp"]["eps_max_approx"]
    assert -0.0312 < lo < -0.0311 and 0.0283 < hi < 0.0285
    lo_r, hi_r = GOLDEN["fast_exp"]["exponent_range"]
    assert abs(-math.log(255.0) - lo_r) < 1e-3 and hi_r == 0.0
    # the skip test must be made on P: exp^(-ln 255) falls below 1/255
    assert float(oracle.fast_exp(-math.log(255.0))) < 1.0 / 255.0
    assert float(oracle.fast_exp(0.0)) < 1.0


@settings(max_examples=300, deadline=None)
@given(st.lists(st.tuples(st.floats(-math.log(255.0), 0.0), st.floats(0.0, 2.0)), min_size=1,
                max_size=60))
def test_fast_exp_colour_bound(pairs):
    """Per-pixel bound: |C^ - C| <= eps/(1-eps) c_max (1 - T^_final) when both blend the same pairs."""
    P = np.array([p for p, _ in pairs])
    c = np.array([cc for _, cc in pairs])
    a = np.minimum(0.99, np.exp(P))
    ah = np.minimum(0.99, oracle.fast_exp(P).astype(np.float64))
    C = Ch = 0.0
    T = Th = 1.0
    for k in range(len(P)):
        if T * (1 - a[k]) < 1e-4 or Th * (1 - ah[k]) < 1e-4:
            if (T * (1 - a[k]) < 1e-4) != (Th * (1 - ah[k]) < 1e-4):
                return                         # a stop flip: outside the bound's premise
            break
        C += a[k] * T * c[k]
        T *= 1 - a[k]
        Ch += ah[k] * Th * c[k]
        Th *= 1 - ah[k]
    eps = FASTEXP.eps_star()
    bound = eps / (1 - eps) * c.max() * (1 - Th)
    assert abs(Ch - C) <= bound + 1e-12


# ---- coefficient folding and the dual pixel (Eqs. expand, c0, coeff, dot, dual_pixel) ------------

def test_folded_coefficients_identity():
    """Eq. dot with Eq. coeff equals p + ln o of Eq. power when b is twice the off-diagonal
    of the conic, and Eq. dual_pixel gives P(x, y+1) exactly."""
    rng = np.random.default_rng(2)
    for _ in range(2000):
        L = rng.normal(size=(2, 2))
        S = L @ L.T + 0.3 * np.eye(2)
        A, B, C = np.linalg.inv(S)[0, 0], np.linalg.inv(S)[0, 1], np.linalg.inv(S)[1, 1]
        u, v = rng.uniform(-20, 20, 2)
        lno = math.log(rng.uniform(0.01, 1))
        x, y = rng.uniform(-10, 10, 2)
        direct = -0.5 * (A * (x - u) ** 2 + C * (y - v) ** 2) - B * (x - u) * (y - v) + lno
        a, b, c = A, 2 * B, C
        C0 = a * u * u + b * u * v + c * v * v
        C1, C2, C3 = -0.5 * a, -0.5 * b, -0.5 * c
        C4, C5, C6 = a * u + 0.5 * b * v, c * v + 0.5 * b * u, -0.5 * C0 + lno
        P = C1 * x * x + C2 * x * y + C3 * y * y + C4 * x + C5 * y + C6
        assert abs(P - direct) <= 1e-9 * (1 + abs(C0))
        P1 = P + C2 * x + C3 * (2 * y + 1) + C5
        d1 = -0.5 * (A * (x - u) ** 2 + C * (y + 1 - v) ** 2) - B * (x - u) * (y + 1 - v) + lno
        assert abs(P1 - d1) <= 1e-9 * (1 + abs(C0))


def _fma32(a, b, c):
    """float32 fused multiply-add: the float64 product of two float32 values is exact."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def test_folded_exponent_never_reaches_the_clamp():
    """The fast rasterizer leaves out alpha's clamp at 0.99.  That is exact only if its float32
    folded exponent P = ln o - q/2 stays below ln(0.99 / exp^(0)) ~ 0.013: q >= 0 and ln o <= 0
    exactly, so this bounds the float32 evaluation error of Eqs. coeff/dot/dual_pixel in
    tile-centre coordinates.  Adversarial sampling: the largest conic the 0.3 dilation allows,
    strongly elongated ones, opacity near 1, means anywhere near the tile."""
    rng = np.random.default_rng(11)
    n = 200_000
    lam1 = 0.3 + rng.exponential(1.0, n) * rng.choice([0.0, 1.0, 100.0], n)
    lam2 = 0.3 + rng.exponential(1.0, n) * rng.choice([0.0, 1.0, 1e4], n)
    th = rng.uniform(0, np.pi, n)
    cs, sn = np.cos(th), np.sin(th)
    S00 = lam1 * cs * cs + lam2 * sn * sn
    S11 = lam1 * sn * sn + lam2 * cs * cs
    S01 = (lam1 - lam2) * cs * sn
    det = S00 * S11 - S01 * S01
    A = (S11 / det).astype(np.float32)
    B = (-S01 / det).astype(np.float32)
    C = (S00 / det).astype(np.float32)
    u = rng.uniform(-9.0, 9.0, n).astype(np.float32)
    v = rng.uniform(-9.0, 9.0, n).astype(np.float32)
    lno = (-rng.exponential(1e-3, n)).astype(np.float32)
    # the pixel pair of a lane: x in -7.5..7.5, y in -7.5, -5.5, ..., 6.5 and y + 1
    x = (rng.integers(0, 16, n) - 7.5).astype(np.float32)
    y = (2 * rng.integers(0, 8, n) - 7.5).astype(np.float32)
    # put half of the pixels right at the mean, where P is largest
    at = rng.random(n) < 0.5
    u = np.where(at, x + rng.uniform(-0.5, 0.5, n).astype(np.float32), u).astype(np.float32)
    v = np.where(at, y + rng.uniform(-0.5, 1.5, n).astype(np.float32), v).astype(np.float32)
    f32 = np.float32
    C0 = _fma32(A * u, u, _fma32(f32(2.0) * B * u, v, C * v * v))
    a_x, a_y, a_z = f32(-0.5) * A, -B, f32(-0.5) * C
    a_w = _fma32(A, u, B * v)
    m_x = _fma32(C, v, B * u)
    m_y = _fma32(np.full(n, -0.5, f32), C0, lno)
    x2, xy, y2 = x * x, x * y, y * y
    y21 = _fma32(np.full(n, 2.0, f32), y, np.ones(n, f32))
    P0 = _fma32(a_x, x2, _fma32(a_y, xy, _fma32(a_z, y2, _fma32(a_w, x, _fma32(m_x, y, m_y)))))
    P1 = P0 + _fma32(a_y, x, _fma32(a_z, y21, m_x))
    top = float(max(P0.max(), P1.max()))
    assert top < 1e-3
    assert float(oracle.fast_exp(top)) < 0.978


# ---- the exact ellipse-tile test (an extension of the Sec. IV-A culling step) -----------------

def _dense_min_q(u, v, c00, c01, c11, det, X0, Y0, n=161):
    """Least q over an n x n grid of the box [X0, X0+15] x [Y0, Y0+15], corners included."""
    xs = np.linspace(X0, X0 + 15.0, n)
    ys = np.linspace(Y0, Y0 + 15.0, n)
    dx = xs[None, :] - u
    dy = ys[:, None] - v
    q = (c11 * dx * dx - 2.0 * c01 * dx * dy + c00 * dy * dy) / det
    return float(q.min())


def test_exact_tile_test_against_dense_sampling():
    """The closed-form edge minimum against brute force: a kept tile has a sampled point
    with q within sampling error of tau, a dropped tile has none below tau; pixel centres
    with alpha >= 1/255 never sit in a dropped tile."""
    rng = np.random.default_rng(5)
    checked = dropped = 0
    for _ in range(3000):
        L = rng.normal(size=(2, 2)) * rng.choice([1.0, 3.0, 10.0])
        S = L @ L.T + 0.3 * np.eye(2)
        c00, c01, c11 = S[0, 0], S[0, 1], S[1, 1]
        det = c00 * c11 - c01 * c01
        tau = 2.0 * (math.log(255.0) + math.log(rng.uniform(1.0 / 255.0, 1.0)))
        u, v = rng.uniform(-40.0, 56.0, 2)
        tx, ty = 0, 0
        keep = bool(oracle.ellipse_meets_tile(u, v, c00, c01, c11, det, tau, tx, ty))
        qmin = _dense_min_q(u, v, c00, c01, c11, det, 0.0, 0.0)
        # pixel centres of the tile
        px, py = np.meshgrid(np.arange(16.0), np.arange(16.0))
        qpix = (c11 * (px - u) ** 2 - 2.0 * c01 * (px - u) * (py - v) + c00 * (py - v) ** 2) / det
        if not keep:
            dropped += 1
            assert qpix.min() > tau
            assert qmin > tau
        if abs(qmin - tau) > 0.02 * tau + 0.05:      # away from the boundary the sampling decides
            checked += 1
            assert keep == (qmin <= tau), (u, v, S.tolist(), tau, qmin)
    assert checked > 2000 and dropped > 300


def test_exact_tiles_change_entries_not_the_image():
    """Dropped tiles hold no pixel with alpha >= 1/255: the entries shrink, the image does not change."""
    sc = wl.config_scene("small", n=3000)
    cam = wl.config_camera("small")
    arr = oracle.prepare_fast(oracle.quantize_scene(sc))
    a = oracle.render(arr, cam, "fast", modes=("fast-def", "fast-exact"))
    b = oracle.render(arr, cam, "fast", modes=("fast-def", "fast-exact"), exact_tiles=True)
    assert b.keys.size < 0.95 * a.keys.size
    for m in ("fast-def", "fast-exact"):
        assert np.array_equal(a.images[m], b.images[m])
    # the kept entries are a subset, in the same emission order
    ka = list(zip(a.entry_gauss.tolist(), a.entry_tile.tolist()))
    kb = list(zip(b.entry_gauss.tolist(), b.entry_tile.tolist()))
    it = iter(ka)
    assert all(e in it for e in kb)


def test_exact_tiles_keep_large_rectangles():
    """Rectangles of more than 64 tiles keep every tile, even those the ellipse misses."""
    plan = oracle.frame_plan(320, 320)
    # a thin diagonal ellipse spanning a 9 x 9 tile rectangle
    c00 = c11 = 2000.0
    c01 = 1999.0
    det = c00 * c11 - c01 * c01
    rect = np.array([[0, 8, 0, 8]])
    eg, et = oracle.duplicate(rect, np.array([True]), plan)
    args = (rect, np.array([72.0]), np.array([72.0]), np.array([[c00, c01, c11]]), np.array([det]),
            np.array([0.0]), plan)
    g, t = oracle.exact_tile_filter(eg, et, *args)
    assert g.size == 81
    meets = oracle.ellipse_meets_tile(72.0, 72.0, c00, c01, c11, det, 2.0 * math.log(255.0),
                                      et % plan.tiles_x, et // plan.tiles_x)
    assert 0 < int(meets.sum()) < 81
    # the same ellipse in a rectangle of 8 x 8 tiles is filtered
    rect8 = np.array([[0, 7, 0, 7]])
    eg8, et8 = oracle.duplicate(rect8, np.array([True]), plan)
    g8, _ = oracle.exact_tile_filter(eg8, et8, rect8, *args[1:])
    assert 0 < g8.size < 64


# ---- paths agree where the paper says they must -----------------------------------------------

def test_plain_equals_fast_exact_on_unquantised_scene():
    """Without quantisation and without depth-bin ties, the fast path's culling and
    32-bit key change nothing: the images agree (Sec. IV-A, Eq. depth_quant)."""
    sc = wl.config_scene("small", n=1500)
    cam = wl.config_camera("small")
    arr = oracle.prepare_plain(sc)
    fr_p = oracle.render(arr, cam, "plain")
    arr_f = dict(arr)
    arr_f["log_opacity"] = np.log(arr_f.pop("opacity"))
    fr_f = oracle.render(arr_f, cam, "fast", modes=("fast-exact",))
    # no two Gaussians of one tile share a depth bin
    k = fr_f.sorted_keys
    assert not np.any(k[1:] == k[:-1])
    assert fr_f.keys.size < fr_p.keys.size                # opacity culling shrinks the tile sets
    assert np.max(np.abs(fr_f.image - fr_p.image)) < 1e-12


def test_oracle_invariants_small_subset():
    sc = wl.config_scene("small", n=2000)
    cam = wl.config_camera("small")
    fr = oracle.render(oracle.prepare_plain(sc), cam, "plain")
    assert np.all((fr.T_final >= 0) & (fr.T_final <= 1))
    assert np.all(fr.image >= 0)
    assert np.all(fr.image <= fr.c_max[None] * (1 - fr.T_final[None]) + 1e-12)
    assert np.all(fr.n_proc <= np.max(fr.ranges[:, 1] - fr.ranges[:, 0]))
