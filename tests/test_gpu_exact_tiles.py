"""The fast path with the exact ellipse-tile test (RGS_EXACT_TILES), through the
C ABI, against the oracle's fast path with the same test (needs an MI355X).
Bars of the fast path: front-end values and entries bit-exact, image within
the fast-exp bound."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from parity import compare_entries, compare_front_end, compare_image, oracle_frame_ablated

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


def run(R, scene, cam, ablations=(), tiles=None):
    path = "/".join(["fast"] + ["no-" + a for a in ablations] + ["exact-tiles"])
    _log(f"[exact-tiles] {path} n={scene.n} {cam.width}x{cam.height}")
    ds = R.upload(scene, ("plain", "fast"))
    g = R.render_debug(ds, cam, path)
    ds.release()
    fr = oracle_frame_ablated(scene, cam, ablations, tiles=tiles, exact_tiles=True)
    compare_front_end(g, fr)
    compare_entries(g, fr)
    rep = compare_image(g["image"], fr, "fast")
    mask = ~fr.flagged & ~(fr.mode_slack > 0) & ~np.isnan(fr.T_final)
    assert np.array_equal(g["n_proc"][mask], fr.n_proc[mask].astype(np.uint32)), "pair counts differ"
    _log(f"[exact-tiles] {path}: entries {g['stats']['n_entries']} {rep}")
    return g, fr


def test_small(R):
    run(R, wl.config_scene("small"), wl.config_camera("small"))


@pytest.mark.parametrize("ablations", [("fusion",), ("key32",), ("fastexp", "dualpixel")])
def test_with_ablations(R, ablations):
    run(R, wl.config_scene("small"), wl.config_camera("small"), ablations)


def test_ragged_frame(R):
    run(R, wl.config_scene("small", n=2500), wl.config_camera("small", width=250, height=170))


def test_fewer_entries_same_image(R):
    """Against the default fast path on the GPU: fewer entries, and the image within the
    bit-level exponential's tolerance (pixels at alpha = 1/255 may be decided differently
    by the float32 skip test and the float64 tile test)."""
    sc = wl.config_scene("small")
    cam = wl.config_camera("small")
    ds = R.upload(sc, ("fast",))
    a = R.render_debug(ds, cam, "fast")
    b = R.render_debug(ds, cam, "fast/exact-tiles")
    ds.release()
    assert b["stats"]["n_entries"] < 0.95 * a["stats"]["n_entries"]
    err = float(np.max(np.abs(a["image"] - b["image"])))
    _log(f"[exact-tiles] entries {a['stats']['n_entries']} -> {b['stats']['n_entries']}, max |diff| {err:.2e}")
    assert err < 2e-2
    assert float(np.mean(np.abs(a["image"] - b["image"]) > 1e-6)) < 1e-3


def test_1080p_keys_and_sampled_tiles(R):
    """1M Gaussians at 1920x1080: every key bit-exact, image on 32 sampled tiles."""
    sc = wl.config_scene("1080p")
    cam = wl.config_camera("1080p")
    plan = oracle.frame_plan(cam.width, cam.height)
    tiles = np.random.default_rng(9).choice(plan.n_tiles, 32, replace=False)
    run(R, sc, cam, tiles=tiles)
