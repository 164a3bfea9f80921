"""The fast path with each of the paper's optimisations removed, through the
C ABI, against the oracle's fast path with the same step removed (needs an
MI355X).  Same bars as the fast path: front-end values and entries bit-exact,
image within the fast-exp bound (or within 2e-3 of the exact-exp oracle when
the bit-level exponential is the step removed)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as wl
from parity import compare_entries, compare_front_end, compare_image, oracle_frame_ablated

pytestmark = pytest.mark.gpu

ABLATIONS = ["fastexp", "dualpixel", "fusion", "extent", "key32", "int8sh", "fp16geom"]


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


def run(R, scene, cam, ablations):
    path = "fast/" + "/".join("no-" + a for a in ablations)
    _log(f"[ablation] {path} n={scene.n} {cam.width}x{cam.height}")
    ds = R.upload(scene, ("plain", "fast"))
    g = R.render_debug(ds, cam, path)
    ds.release()
    fr = oracle_frame_ablated(scene, cam, ablations)
    compare_front_end(g, fr)
    compare_entries(g, fr)
    rep = compare_image(g["image"], fr, "fast")
    mask = ~fr.flagged & ~(fr.mode_slack > 0) & ~np.isnan(fr.T_final)
    assert np.array_equal(g["n_proc"][mask], fr.n_proc[mask].astype(np.uint32)), "pair counts differ"
    assert np.array_equal(g["n_blend"][mask], fr.n_blend[mask].astype(np.uint32)), "blended counts differ"
    _log(f"[ablation] {path}: entries {g['stats']['n_entries']} {rep}")
    return g


@pytest.mark.parametrize("ablation", ABLATIONS)
def test_each_ablation_matches_its_oracle(R, ablation):
    run(R, wl.config_scene("small"), wl.config_camera("small"), [ablation])


def test_all_ablations_together(R):
    run(R, wl.config_scene("small"), wl.config_camera("small"), ABLATIONS)


@pytest.mark.parametrize("ablation", ["dualpixel", "fusion", "key32"])
def test_ragged_frame(R, ablation):
    run(R, wl.config_scene("small", n=2500), wl.config_camera("small", width=250, height=170), [ablation])


def test_unfused_front_end_is_the_fused_one(R):
    """Fusion changes where the front end's work happens, not its results."""
    sc = wl.config_scene("small")
    cam = wl.config_camera("small")
    ds = R.upload(sc, ("plain", "fast"))
    a = R.render_debug(ds, cam, "fast")
    b = R.render_debug(ds, cam, "fast/no-fusion")
    ds.release()
    for k in ("image", "keys_unsorted", "vals_unsorted", "keys_sorted", "vals_sorted", "ranges", "n_proc"):
        assert np.array_equal(a[k], b[k]), k
