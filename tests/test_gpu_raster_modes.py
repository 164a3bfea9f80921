"""The fast rasterizer's production and counting renders, and its
pixels-per-lane variants, through the C ABI (needs an MI355X).

A production render and a counting (debug) render take the same operations in
the same order (the counting render only adds per-pixel counters), so their
images must agree bit for bit, in scenes where no pixel stops and in scenes
where many do.  The four-pixel variant (Eq. dual_pixel applied along the
column, one wave per tile) is checked against the oracle like the fast path."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as wl
from parity import compare_entries, compare_front_end, compare_image, oracle_frame

pytestmark = pytest.mark.gpu

PATHS = ["fast", "fast/no-fastexp", "fast/no-dualpixel", "fast/no-fastexp/no-dualpixel", "fast/hw-exp2",
         "fast/quad-pixel"]


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


def _stopping_scene():
    return wl.make_scene(4000, 1.0, -2.8, 0.4, 21)      # large Gaussians: many pixels reach T < 1e-4


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("case", ["small", "stopping", "ragged"])
def test_production_equals_counting_render(R, path, case):
    import torch
    if case == "small":
        sc, cam = wl.config_scene("small"), wl.config_camera("small")
    elif case == "stopping":
        sc, cam = _stopping_scene(), wl.config_camera("small", width=160, height=120)
    else:
        sc, cam = wl.config_scene("small", n=2500), wl.config_camera("small", width=250, height=170)
    _log(f"[modes] {path} {case} n={sc.n} {cam.width}x{cam.height}")
    ds = R.upload(sc, ("plain", "fast"))
    img, _ = R.render(ds, cam, path)
    torch.cuda.synchronize()
    prod = img.cpu().numpy().copy()
    g = R.render_debug(ds, cam, path)
    ds.release()
    stopped = int(np.count_nonzero(g["stopped"]))
    _log(f"[modes] {path} {case}: {stopped} pixels stopped")
    if case == "stopping":
        assert stopped > 100
    assert np.array_equal(prod.view(np.uint32), g["image"].view(np.uint32)), \
        f"production and counting renders differ at {int(np.count_nonzero(prod != g['image']))} values"


@pytest.mark.parametrize("case", ["small", "stopping", "ragged"])
def test_quad_pixel_against_oracle(R, case):
    if case == "small":
        sc, cam = wl.config_scene("small"), wl.config_camera("small")
    elif case == "stopping":
        sc, cam = _stopping_scene(), wl.config_camera("small", width=160, height=120)
    else:
        sc, cam = wl.config_scene("small", n=2500), wl.config_camera("small", width=250, height=170)
    _log(f"[quad] {case} n={sc.n} {cam.width}x{cam.height}")
    ds = R.upload(sc, ("fast",))
    g = R.render_debug(ds, cam, "fast/quad-pixel")
    ds.release()
    fr = oracle_frame(sc, cam, "fast")
    compare_front_end(g, fr)
    compare_entries(g, fr)
    rep = compare_image(g["image"], fr, "fast")
    mask = ~fr.flagged & ~(fr.mode_slack > 0) & ~np.isnan(fr.T_final)
    assert np.array_equal(g["n_proc"][mask], fr.n_proc[mask].astype(np.uint32)), "pair counts differ"
    assert np.array_equal(g["n_blend"][mask], fr.n_blend[mask].astype(np.uint32)), "blended counts differ"
    _log(f"[quad] {case}: {rep}")
