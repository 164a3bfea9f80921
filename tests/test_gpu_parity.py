"""HIP renderer against the FP64 oracle through the C ABI (needs an MI355X)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from parity import compare_entries, compare_front_end, compare_image, oracle_frame

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


ORDER_CHUNK, ORDER_CLASSES, ORDER_MAX_TILES = 8192, 32, 16384


def check_tile_order(order, ranges, path):
    """The rasterizers' schedule.  Plain-path frames and fast-path frames of at most 16384
    tiles: within each chunk of 8192 tiles a permutation of the chunk, longest lists first
    up to one class width (a 32nd of the chunk's longest).  Other frames: row-major."""
    if not (path.startswith("plain") or len(ranges) <= ORDER_MAX_TILES):
        assert np.array_equal(order, np.arange(len(ranges))), "expected the row-major schedule"
        return
    lengths = ranges[:, 1].astype(np.int64) - ranges[:, 0].astype(np.int64)
    for c0 in range(0, len(ranges), ORDER_CHUNK):
        c1 = min(c0 + ORDER_CHUNK, len(ranges))
        o = order[c0:c1].astype(np.int64)
        assert np.array_equal(np.sort(o), np.arange(c0, c1)), f"chunk {c0}: not a permutation"
        L = lengths[o]
        width = (L.max() + 1) / ORDER_CLASSES
        later_max = np.maximum.accumulate(L[::-1])[::-1]
        assert np.all(later_max[1:] <= L[:-1] + width + 1), f"chunk {c0}: a longer list is scheduled later"


def run_parity(R, scene, cam, path, tiles=None, entries=True):
    _log(f"[parity] path={path} n={scene.n} {cam.width}x{cam.height} tiles={'all' if tiles is None else len(tiles)}")
    ds = R.upload(scene, (path,))
    g = R.render_debug(ds, cam, path)
    ds.release()
    check_tile_order(g["tile_order"], g["ranges"], path)
    fr = oracle_frame(scene, cam, path, tiles=tiles)
    compare_front_end(g, fr)
    if entries:
        compare_entries(g, fr)
    rep = compare_image(g["image"], fr, path)
    rep.update(n_entries=int(g["stats"]["n_entries"]), n_visible=int(g["stats"]["n_visible"]),
               max_tile_entries=int((g["ranges"][:, 1].astype(np.int64) - g["ranges"][:, 0]).max()))
    # pair evaluations agree with the oracle's count except where a decision was flagged
    mask = ~fr.flagged & ~(fr.mode_slack > 0) & ~np.isnan(fr.T_final)
    assert np.array_equal(g["n_proc"][mask], fr.n_proc[mask].astype(np.uint32)), "pair counts differ"
    assert np.array_equal(g["n_blend"][mask], fr.n_blend[mask].astype(np.uint32)), "blended counts differ"
    _log(f"[parity] {path}: {rep}")
    return rep


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_small_full(R, path):
    run_parity(R, wl.config_scene("small"), wl.config_camera("small"), path)


@pytest.mark.parametrize("path", ["plain", "fast"])
@pytest.mark.parametrize("W,H", [(250, 170), (17, 33), (1, 1), (64, 16)])
def test_ragged_sizes(R, path, W, H):
    run_parity(R, wl.config_scene("small", n=2500), wl.config_camera("small", width=W, height=H), path)


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_background_and_termination(R, path):
    sc = wl.make_scene(4000, 1.0, -2.8, 0.4, 21)        # larger Gaussians: many pixels stop early
    cam = wl.config_camera("small", width=160, height=120)
    cam.bg = np.array([0.2, 0.5, 0.7], np.float32)
    rep = run_parity(R, sc, cam, path)
    assert rep["n_entries"] > 0


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_empty_frame(R, path):
    import torch
    sc = wl.config_scene("small", n=500)
    cam = wl.look_at_camera((0, 0, 30.0), (0, 0, 40.0), (0, 1, 0), 60.0, 48, 40, 1.0, 2.0,
                            bg=(0.1, 0.2, 0.3))
    ds = R.upload(sc, (path,))
    img, st = R.render(ds, cam, path)
    torch.cuda.synchronize()
    assert st["n_entries"] == 0 and st["n_visible"] == 0
    expect = np.broadcast_to(np.array([0.1, 0.2, 0.3], np.float32)[:, None, None], (3, 40, 48))
    assert np.array_equal(img.cpu().numpy(), expect)


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_equal_keys_keep_index_order(R, path):
    """Many copies of a few Gaussians: long runs of equal keys must end up in index order."""
    base = wl.config_scene("small", n=40)
    idx = np.tile(np.arange(40), 150)
    sc = base.subset(idx)
    run_parity(R, sc, wl.config_camera("small", width=128, height=96), path)


@pytest.mark.parametrize("copies", [4000, 7000])
def test_bucket_larger_than_lds(R, copies):
    """Copies of 40 Gaussians at 256x256.  The frame has 256 tiles, so each of the fast sort's
    buckets holds one tile, and the most covered tiles get more entries than the LDS holds
    (16384): with 4000 copies 20000 each, sorted as two runs in LDS and merged; with 7000
    copies 35000 each, more than two runs, streamed through global memory in chunks.  Keys,
    values and ranges bit-exact (with long runs of equal keys), the image on 12 tiles."""
    base = wl.config_scene("small", n=40)
    sc = base.subset(np.tile(np.arange(40), copies))
    cam = wl.config_camera("small", width=256, height=256)
    plan = oracle.frame_plan(cam.width, cam.height)
    tiles = np.random.default_rng(5).choice(plan.n_tiles, 12, replace=False)
    rep = run_parity(R, sc, cam, "fast", tiles=tiles)
    assert rep["max_tile_entries"] > (16384 if copies == 4000 else 2 * 16384), rep


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_deterministic(R, path):
    import torch
    sc = wl.config_scene("small")
    cam = wl.config_camera("small")
    ds = R.upload(sc, (path,))
    a = R.render_debug(ds, cam, path)
    b = R.render_debug(ds, cam, path)
    for k in ("image", "keys_sorted", "vals_sorted", "ranges", "n_proc"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_capacity_overflow_is_reported(R, path):
    import paper_2608_15785_amd as rgs
    import torch
    sc = wl.config_scene("small")
    cam = wl.config_camera("small")
    ds = R.upload(sc, (path,))
    ws = rgs.new_workspace(sc.n, cam.width, cam.height, path, 1000)
    with pytest.raises(rgs.RGSError) as e:
        rgs.render(R.ctx, ds, cam, path, ws, stats=True)
    assert e.value.status == -4
    from paper_2608_15785_amd._binding import workspace_stats
    st = workspace_stats(R.ctx, ws, sc.n)
    assert st["overflow"] == 1 and 1000 <= st["capacity"] < st["n_entries"]
    # the renderer grows its workspace and the frame then matches the oracle
    img, st = R.render(ds, cam, path)
    assert st["overflow"] == 0


def test_invalid_arguments(R):
    import paper_2608_15785_amd as rgs
    sc = wl.config_scene("small", n=100)
    ds = R.upload(sc, ("fast",))
    cam = wl.config_camera("small")
    ws = rgs.new_workspace(sc.n, 256, 256, "plain", 10000)
    with pytest.raises(rgs.RGSError) as e:          # plain path on a fast-only scene
        rgs.render(R.ctx, ds, cam, "plain", ws)
    assert e.value.status == -1
    bad = wl.config_camera("small")
    bad.z_near, bad.z_far = 3.0, 2.0
    with pytest.raises(rgs.RGSError):
        rgs.render(R.ctx, ds, bad, "fast", ws)
    bad = wl.config_camera("small")
    bad.width = 0
    with pytest.raises(rgs.RGSError):
        rgs.render(R.ctx, ds, bad, "fast", ws)
    bad = wl.config_camera("small")
    bad.height = 20000
    with pytest.raises(rgs.RGSError):
        rgs.render(R.ctx, ds, bad, "fast", ws)


def test_sizing_by_scene(R):
    """rgs_render_workspace_bound is rgs_workspace_size with the scene's n (and a default
    entry guess), and rgs_scene_device_bytes is rgs_scene_info's byte count."""
    import paper_2608_15785_amd as rgs
    from paper_2608_15785_amd import _binding as B
    sc = wl.config_scene("small", n=3000)
    ds = R.upload(sc, ("plain", "fast"))
    assert ds.device_bytes() == ds.info()["device_bytes"] > 0
    for path in ("fast", "plain"):
        assert ds.workspace_bound(1920, 1080, path, 12345) == B.workspace_size(sc.n, 1920, 1080, path, 12345)
        assert ds.workspace_bound(1920, 1080, path) == B.workspace_size(sc.n, 1920, 1080, path, 65536)
        bound = ds.workspace_bound(256, 256, path, 50000)
        assert B.workspace_capacity(sc.n, 256, 256, path, bound) >= 50000
    with pytest.raises(rgs.RGSError):
        ds.workspace_bound(0, 1080, "fast")
    with pytest.raises(rgs.RGSError):
        ds.workspace_bound(1920, 1080, "fast", B.MAX_ENTRIES + 1)
    ds.release()


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_1080p_keys_and_sampled_tiles(R, path):
    """1M Gaussians at 1920x1080: every key bit-exact, image on 64 sampled tiles."""
    sc = wl.config_scene("1080p")
    cam = wl.config_camera("1080p")
    plan = oracle.frame_plan(cam.width, cam.height)
    tiles = np.random.default_rng(7).choice(plan.n_tiles, 64, replace=False)
    tiles = np.concatenate([tiles, [plan.n_tiles - 1]])          # the ragged corner tile
    run_parity(R, sc, cam, path, tiles=tiles)


@pytest.mark.parametrize("path", ["plain", "fast"])
@pytest.mark.parametrize("pose", [0, 8, 16, 21, 32, 40, 48, 56])
def test_4k_keys_and_sampled_tiles(R, path, pose):
    """3M Gaussians at 3840x2160 on eight orbit poses: every key bit-exact, 24 sampled tiles each."""
    sc = _4k_scene()
    cam = wl.config_camera("4k", pose=pose)
    plan = oracle.frame_plan(cam.width, cam.height)
    tiles = np.random.default_rng(pose).choice(plan.n_tiles, 24, replace=False)
    run_parity(R, sc, cam, path, tiles=tiles)


@pytest.mark.parametrize("path", ["plain", "fast"])
@pytest.mark.parametrize("W,H", [(2560, 1440), (2048, 2048)])
def test_two_schedule_chunks_keys_and_sampled_tiles(R, path, W, H):
    """The 1M scene at 2560x1440 (14400 tiles) and 2048x2048 (16384, the most the fast path's
    bucket sort and tile schedule take): b_t = 14, 64 tiles per bucket, and the schedule in two
    chunks of 8192 tiles.  Every key bit-exact, the order checked, 32 sampled tiles and the last."""
    sc = wl.config_scene("1080p")
    cam = wl.config_camera("1080p", width=W, height=H)
    plan = oracle.frame_plan(cam.width, cam.height)
    assert plan.b_t == 14 and ORDER_CHUNK < plan.n_tiles <= ORDER_MAX_TILES
    tiles = np.concatenate([np.random.default_rng(W + H).choice(plan.n_tiles, 32, replace=False),
                            [plan.n_tiles - 1]])
    run_parity(R, sc, cam, path, tiles=tiles)


@pytest.mark.parametrize("path", ["plain", "fast"])
@pytest.mark.parametrize("pose", [0, 37])
def test_720p_keys_and_sampled_tiles(R, path, pose):
    """The serving mix's 1280x720 class (half of its requests): the 1M scene on its serving
    orbit, every key bit-exact, 48 sampled tiles and the ragged last tile."""
    sc = wl.config_scene("1080p")
    cam = wl.serving_camera(0, pose, 1280, 720)
    plan = oracle.frame_plan(cam.width, cam.height)
    tiles = np.concatenate([np.random.default_rng(72 + pose).choice(plan.n_tiles, 48, replace=False),
                            [plan.n_tiles - 1]])
    run_parity(R, sc, cam, path, tiles=tiles)


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_largest_frame(R, path):
    """The largest accepted frame, 16384x16384: 2^20 tiles, so the fast key keeps only
    12 depth bits and many keys tie.  Every key and range bit-exact; the image on 16
    random tiles, nine tiles around the centre and the four corners."""
    cam = wl.config_camera("small", width=16384, height=16384)
    plan = oracle.frame_plan(cam.width, cam.height)
    assert plan.b_t == 20 and plan.b_d == 12
    tx0, ty0 = plan.tiles_x // 2, plan.tiles_y // 2
    centre = [(ty0 + dy) * plan.tiles_x + tx0 + dx for dy in (-2, 0, 2) for dx in (-2, 0, 2)]
    corners = [0, plan.tiles_x - 1, plan.n_tiles - plan.tiles_x, plan.n_tiles - 1]
    tiles = np.concatenate([np.random.default_rng(11).choice(plan.n_tiles, 16, replace=False), centre, corners])
    run_parity(R, wl.config_scene("small", n=2000), cam, path, tiles=tiles)


@pytest.mark.parametrize("path", ["plain", "fast"])
@pytest.mark.parametrize("n", [1, 65, 1025, 256 * 4096, 256 * 4096 + 1])
def test_front_end_block_shapes(R, path, n):
    """Scene sizes at the edges of how the front end splits Gaussians over workgroups:
    one Gaussian, a count just past a multiple of 64 and past 1024, exactly 256 full
    workgroups of 4096 (the even split) and one more (4096 per workgroup).  Every key
    bit-exact; the image on 8 sampled tiles of the small frame."""
    cam = wl.config_camera("small")
    plan = oracle.frame_plan(cam.width, cam.height)
    tiles = None if n < 100_000 else np.random.default_rng(n % 97).choice(plan.n_tiles, 8, replace=False)
    run_parity(R, wl.config_scene("small", n=n), cam, path, tiles=tiles)


_CFG2 = {}


def _4k_scene():
    if "s" not in _CFG2:
        _CFG2["s"] = wl.config_scene("4k")
    return _CFG2["s"]


@pytest.mark.parametrize("path", ["plain", "fast"])
def test_sort_fallback_counts_match(R, path):
    """Every radix tile counting its predecessors from their keys (the look-back's fallback,
    forced with the context's RGS_DEBUG_SORT_FALLBACK) gives the same bit-exact entries, at
    1M / 1080p and on the small frame."""
    from paper_2608_15785_amd import _binding as B
    R.ctx.set_debug(B.DEBUG_SORT_FALLBACK)
    try:
        run_parity(R, wl.config_scene("small"), wl.config_camera("small"), path)
        sc = wl.config_scene("1080p")
        cam = wl.config_camera("1080p")
        plan = oracle.frame_plan(cam.width, cam.height)
        tiles = np.random.default_rng(3).choice(plan.n_tiles, 16, replace=False)
        run_parity(R, sc, cam, path, tiles=tiles)
    finally:
        R.ctx.set_debug(0)
