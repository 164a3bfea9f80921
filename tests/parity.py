"""Comparison of the HIP renderer with the FP64 oracle on the same seeded inputs.

Bars (see the oracle's blend module for the decision bookkeeping):
* per-Gaussian visibility, tile rectangle and float64 depth, mean and 2D
  covariance: bit-exact;
* duplicated entries in emission order, sorted keys and indices, tile ranges:
  bit-exact;
* plain image: |gpu - oracle| <= 2e-3 + slack at every pixel;
* fast image: |gpu - oracle(bit-level exp)| <= 1e-4 at every pixel whose
  decisions all lie outside the float32 margins, <= 2e-3 + slack at the
  flagged ones, and |gpu - oracle(exact exp)| <= eps/(1-eps) c_max
  (1 - T_final) + 1e-3 + slack (the per-pixel bound of the bit-level
  exponential, Sec. IV-B), where slack is the colour at stake in skip/stop
  decisions that lie within the float32 margin of their thresholds, or that
  the two exponentials decide differently.  The flagged share of the pixels is
  capped.

Fast-path margins.  A float32 evaluation of the folded exponent (Eqs. expand,
coeff, dot, dual_pixel in tile-centre coordinates) rounds each term it adds,
so its error is bounded by a multiple of M, the sum of the terms' magnitudes
(see the oracle's blend module).  A float32 replica of that arithmetic over 2M
random conics, means and pixels stays within 3.5e-7 M; the margin on P and on
the relative alpha is 4e-6 M per pair (about 12 times that), plus 1e-5 on
alpha for the bit-level exponential's float32 rounding (its integer is a
multiple of 64 at these magnitudes, 5.3e-6 relative), and every blended pair
widens the transmittance interval by one float32 rounding.
"""
from __future__ import annotations

import importlib
import math

import numpy as np

import oracle

FASTEXP = importlib.import_module("oracle.fastexp")

PLAIN_TOL = 2e-3
FAST_TOL = 1e-3
FAST_UNFLAGGED_TOL = 1e-4        # fast image vs the bit-level-exp oracle where no decision is flagged
# most pixels whose fast-path decisions may be flagged: 1.5 % of a comparison of
# at least 4096 pixels (measured 0.2 - 1.1 % on every such case), 5 % below that
FAST_FLAG_CAP = (0.015, 0.05)
PLAIN_MARGINS = (1e-4, 0.0)      # relative alpha uncertainty of float32 + expf
# relative alpha, absolute P, per-pair scale of the terms' magnitudes, float32 rounding of T
FAST_MARGINS = (1e-5, 1e-6, 4e-6, 2.0 ** -22)
# the plain path's training variant: the plain definition (exact exponential,
# alpha = min(0.99, o e^p)) evaluated in the folded form, so the fast path's
# per-pair margins, with M taken in tile-centre coordinates
TRAIN_MARGINS = (1e-5, 0.0, 4e-6, 2.0 ** -22)

_PREPARED = {}


def _prepared(scene, kind):
    """Oracle arrays of a scene ("plain" or "fast"), kept for the scene object."""
    key = (id(scene), kind)
    hit = _PREPARED.get(key)
    if hit is None or hit[0] is not scene:
        arr = oracle.prepare_plain(scene) if kind == "plain" else oracle.prepare_fast(oracle.quantize_scene(scene))
        if len(_PREPARED) > 8:
            _PREPARED.clear()
        _PREPARED[key] = hit = (scene, arr)
    return hit[1]


def oracle_frame(scene, cam, path, tiles=None, workers=8):
    if path == "plain":
        return oracle.render(_prepared(scene, "plain"), cam, "plain", tiles=tiles, margins=PLAIN_MARGINS,
                             workers=workers)
    if path == "plain/hw-exp2":
        return oracle.render(_prepared(scene, "plain"), cam, "plain", tiles=tiles, margins=TRAIN_MARGINS,
                             margin_frame="tile-centre", workers=workers)
    return oracle.render(_prepared(scene, "fast"), cam, "fast", modes=("fast-def", "fast-exact"), tiles=tiles,
                         margins=FAST_MARGINS, workers=workers)


def oracle_frame_ablated(scene, cam, ablations, tiles=None, workers=8, exact_tiles=False):
    """The oracle's fast path with the named steps removed (see the binding's
    ABLATIONS): storage read in FP32, 3-sigma extent, 64-bit key, exact exp;
    with ``exact_tiles`` it adds the exact ellipse-tile test."""
    ab = set(ablations)
    fs = oracle.quantize_scene(scene)
    arr = oracle.prepare_fast_ablated(scene, fs, int8_sh="int8sh" not in ab, fp16_geometry="fp16geom" not in ab)
    modes = ("fast-exact",) if "fastexp" in ab else ("fast-def", "fast-exact")
    return oracle.render(arr, cam, "fast", modes=modes, tiles=tiles, margins=FAST_MARGINS, workers=workers,
                         alpha_extent="extent" not in ab, key64="key32" in ab, exact_tiles=exact_tiles)


def compare_front_end(g, fr):
    vis = fr.proj.visible
    assert np.array_equal(g["visible"], vis), f"visibility differs at {np.nonzero(g['visible'] != vis)[0][:10]}"
    assert np.array_equal(g["depth"].view(np.uint64), fr.proj.d.view(np.uint64)), "depth bits differ"
    for k, ref in (("u", fr.proj.u), ("v", fr.proj.v)):
        assert np.array_equal(g[k][vis].view(np.uint64), ref[vis].view(np.uint64)), f"{k} bits differ"
    assert np.array_equal(g["cov2d"][vis].view(np.uint64), fr.proj.cov[vis].view(np.uint64)), "cov2d bits differ"
    assert np.array_equal(g["rect"][vis].astype(np.int64), fr.proj.rect[vis]), "tile rectangles differ"
    cerr = float(np.max(np.abs(g["color"][vis] - fr.proj.color[vis]))) if vis.any() else 0.0
    assert cerr < 1e-5, f"SH colour differs by {cerr}"
    return cerr


def compare_entries(g, fr):
    assert g["stats"]["n_entries"] == fr.keys.size, (g["stats"]["n_entries"], fr.keys.size)
    assert np.array_equal(g["keys_unsorted"], fr.keys), "unsorted keys differ"
    assert np.array_equal(g["vals_unsorted"].astype(np.int64), fr.entry_gauss), "unsorted indices differ"
    assert np.array_equal(g["keys_sorted"], fr.sorted_keys), "sorted keys differ"
    assert np.array_equal(g["vals_sorted"].astype(np.int64), fr.sorted_gauss), "sorted indices differ"
    assert np.array_equal(g["ranges"].astype(np.int64), fr.ranges), "tile ranges differ"


def _tile_mask(fr):
    H, W = fr.plan.height, fr.plan.width
    m = np.zeros((H, W), bool)
    for t in fr.tiles:
        tx, ty = int(t) % fr.plan.tiles_x, int(t) // fr.plan.tiles_x
        m[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = True
    return m


def psnr(a, b, mask=None):
    d = (a - b) if mask is None else (a - b)[:, mask]
    mse = float(np.mean(d * d))
    return math.inf if mse == 0 else 10 * math.log10(1.0 / mse)


def compare_image(img, fr, path):
    """Asserts the image bars on the oracle's blended tiles; returns a report dict."""
    mask = _tile_mask(fr)
    gpu = img[:, mask].astype(np.float64)
    slack = fr.slack[mask][None]
    rep = dict(pixels=int(mask.sum()), flagged=int(fr.flagged[mask].sum()))
    if path == "plain":
        ref = fr.images["plain"][:, mask]
        err = np.abs(gpu - ref)
        bad = err > PLAIN_TOL + slack
        rep.update(max_err=float(err.max()), psnr=psnr(gpu, ref),
                   max_err_unflagged=float(err[:, ~fr.flagged[mask]].max()) if (~fr.flagged[mask]).any() else 0.0)
        assert not bad.any(), f"plain: {int(bad.sum())} values over tolerance, worst {float((err - PLAIN_TOL - slack).max())}"
        return rep
    if "fast-def" not in fr.images:
        # the exponential ablated: the exact-exp oracle is the definition
        ref = fr.images["fast-exact"][:, mask]
        err = np.abs(gpu - ref)
        bad = err > PLAIN_TOL + slack
        assert not bad.any(), f"fast, exact exp: {int(bad.sum())} over, worst {float((err - PLAIN_TOL - slack).max())}"
        unflagged = ~fr.flagged[mask]
        err_unflagged = float(err[:, unflagged].max()) if unflagged.any() else 0.0
        assert err_unflagged <= FAST_UNFLAGGED_TOL, f"fast, exact exp, at unflagged pixels: {err_unflagged}"
        rep.update(max_err=float(err.max()), max_err_unflagged=err_unflagged, psnr=psnr(gpu, ref))
        return rep
    ref_def = fr.images["fast-def"][:, mask]
    ref_exact = fr.images["fast-exact"][:, mask]
    err_def = np.abs(gpu - ref_def)
    bad = err_def > PLAIN_TOL + slack
    assert not bad.any(), f"fast vs bit-level-exp oracle: {int(bad.sum())} over, worst {float((err_def - PLAIN_TOL - slack).max())}"
    unflagged = ~fr.flagged[mask]
    share = 1.0 - float(unflagged.mean()) if unflagged.size else 0.0
    err_unflagged = float(err_def[:, unflagged].max()) if unflagged.any() else 0.0
    assert err_unflagged <= FAST_UNFLAGGED_TOL, f"fast vs bit-level-exp oracle at unflagged pixels: {err_unflagged}"
    cap = FAST_FLAG_CAP[0] if unflagged.size >= 4096 else FAST_FLAG_CAP[1]
    assert share <= cap, f"{share:.2%} of the pixels flagged"
    eps = FASTEXP.eps_star()
    bound = eps / (1 - eps) * fr.c_max[mask] * (1 - fr.T_final[mask])
    allowed = bound[None] + FAST_TOL + slack + fr.mode_slack[mask][None]
    err_ex = np.abs(gpu - ref_exact)
    bad = err_ex > allowed
    assert not bad.any(), f"fast vs exact oracle: {int(bad.sum())} over the bound, worst {float((err_ex - allowed).max())}"
    rep.update(max_err_vs_def=float(err_def.max()), max_err_vs_def_unflagged=err_unflagged,
               flagged_share=round(share, 5), max_err_vs_exact=float(err_ex.max()),
               psnr_vs_def=psnr(gpu, ref_def), psnr_vs_exact=psnr(gpu, ref_exact),
               max_bound=float(bound.max()), mode_flagged=int((fr.mode_slack[mask] > 0).sum()))
    return rep
