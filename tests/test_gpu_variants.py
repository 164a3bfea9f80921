"""gfx950 variants of the rasterizers, through the C ABI, against the oracle
(needs an MI355X).  RGS_HW_EXP2 takes alpha = min(0.99, exp2(P log2 e)) from
the hardware exp2 instruction: its image is the exact-exponential oracle's, to
the same 2e-3 bar as the exponential's ablation; front end and entries are the
fast path's, bit-exact.  With the plain path (its training variant: the
dual-pixel rasterizer with folded coefficients and culled lists over the plain
path's records) the image is the plain oracle's, to the plain path's bar, with
decision margins for the folded float32 arithmetic, and every key bit-exact."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as wl
from parity import compare_entries, compare_front_end, compare_image, oracle_frame, oracle_frame_ablated

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_15785_amd as rgs
    return rgs.Renderer(0)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(R, scene, cam, path, exact_tiles=False):
    _log(f"[variant] {path} n={scene.n} {cam.width}x{cam.height}")
    ds = R.upload(scene, ("plain", "fast"))
    g = R.render_debug(ds, cam, path)
    ds.release()
    # the oracle with the exact exponential (the hardware exp2 is exact to an ulp)
    fr = oracle_frame_ablated(scene, cam, ["fastexp"], exact_tiles=exact_tiles)
    compare_front_end(g, fr)
    compare_entries(g, fr)
    rep = compare_image(g["image"], fr, "fast")
    mask = ~fr.flagged & ~(fr.mode_slack > 0) & ~np.isnan(fr.T_final)
    assert np.array_equal(g["n_proc"][mask], fr.n_proc[mask].astype(np.uint32)), "pair counts differ"
    _log(f"[variant] {path}: {rep}")
    return g


def test_hw_exp2_small(R):
    run(R, wl.config_scene("small"), wl.config_camera("small"), "fast/hw-exp2")


def test_hw_exp2_ragged(R):
    run(R, wl.config_scene("small", n=2500), wl.config_camera("small", width=250, height=170), "fast/hw-exp2")


def test_hw_exp2_with_exact_tiles(R):
    run(R, wl.config_scene("small"), wl.config_camera("small"), "fast/hw-exp2/exact-tiles", exact_tiles=True)


def test_hw_exp2_close_to_exact_exp_ablation(R):
    """The hardware exp2 and the accurate expf give the same image to float32 rounding."""
    sc = wl.config_scene("small")
    cam = wl.config_camera("small")
    ds = R.upload(sc, ("plain", "fast"))
    a = R.render_debug(ds, cam, "fast/hw-exp2")
    b = R.render_debug(ds, cam, "fast/no-fastexp")
    ds.release()
    d = np.abs(a["image"] - b["image"])
    _log(f"[variant] hw-exp2 vs expf: max {float(d.max()):.2e}, share > 1e-5: {float(np.mean(d > 1e-5)):.2e}")
    assert float(np.mean(d > 1e-3)) < 1e-3


@pytest.mark.parametrize("case", ["small", "ragged", "1080p"])
def test_plain_hw_exp2_against_the_plain_oracle(R, case):
    import oracle
    tiles = None
    if case == "small":
        sc, cam = wl.config_scene("small"), wl.config_camera("small")
    elif case == "ragged":
        sc, cam = wl.config_scene("small", n=2500), wl.config_camera("small", width=250, height=170)
    else:
        sc, cam = wl.config_scene("1080p"), wl.config_camera("1080p")
        plan = oracle.frame_plan(cam.width, cam.height)
        tiles = np.random.default_rng(17).choice(plan.n_tiles, 32, replace=False)
    _log(f"[variant] plain/hw-exp2 {case} n={sc.n} {cam.width}x{cam.height}")
    ds = R.upload(sc, ("plain",))
    g = R.render_debug(ds, cam, "plain/hw-exp2")
    ds.release()
    fr = oracle_frame(sc, cam, "plain/hw-exp2", tiles=tiles)
    compare_front_end(g, fr)
    compare_entries(g, fr)
    rep = compare_image(g["image"], fr, "plain")
    mask = ~fr.flagged & ~np.isnan(fr.T_final)
    assert np.array_equal(g["n_proc"][mask], fr.n_proc[mask].astype(np.uint32)), "pair counts differ"
    _log(f"[variant] plain/hw-exp2 {case}: {rep}")
