"""One frame of the tile-based forward render, plain or fast (Sec. II-A, III, IV).

The stages run in the paper's order: preprocess (projection, culling, colour),
duplicate with keys, sort, tile ranges, per-tile blending.  The plain path is
the 3DGS baseline (FP32 attributes, 64-bit key, exact exp).  The fast path
renders the compact scene (``quant``), keys on the 32-bit quantised depth and
shrinks each tile set by opacity culling; it blends with the bit-level
exponential ("fast-def") and, beside it, with the exact exponential
("fast-exact") so that tests can apply the paper's per-pixel error bound.
"""
from __future__ import annotations

import multiprocessing as mp
from dataclasses import dataclass, field

import numpy as np

from .blend import blend_tile
from .plan import TILE, FramePlan, frame_plan
from .project import Projection, project
from .quant import FastScene, dequantize_scene
from .tiles import duplicate, exact_tile_filter, fast_keys, plain_keys, sort_entries, tile_ranges


def prepare_plain(scene) -> dict:
    """float64 view of a float32 scene for the plain path."""
    return dict(means=np.asarray(scene.means, np.float64), quats=np.asarray(scene.quats, np.float64),
                scales=np.asarray(scene.scales, np.float64),
                opacity=np.asarray(scene.opacity, np.float64), sh=np.asarray(scene.sh, np.float64))


def prepare_fast(fs: FastScene) -> dict:
    """float64 view of the stored compact scene for the fast path."""
    return dequantize_scene(fs)


def prepare_fast_ablated(scene, fs: FastScene, int8_sh: bool = True, fp16_geometry: bool = True) -> dict:
    """float64 view of the fast path's inputs with a compact-storage step
    ablated (Sec. IV-A, "Compact Attribute Storage"): FP32 SH instead of the
    INT8 ones, and/or FP32 rotation and scale with ln o taken in float64 and
    rounded to float32, instead of their FP16 forms."""
    arr = dequantize_scene(fs)
    if not int8_sh:
        arr["sh"] = np.asarray(scene.sh, np.float64)
    if not fp16_geometry:
        arr["quats"] = np.asarray(scene.quats, np.float64)
        arr["scales"] = np.asarray(scene.scales, np.float64)
        lno = np.log(np.asarray(scene.opacity, np.float64)).astype(np.float32)
        arr["log_opacity"] = lno.astype(np.float64)
    return arr


@dataclass
class OracleFrame:
    plan: FramePlan
    path: str
    modes: tuple
    proj: Projection
    entry_gauss: np.ndarray      # emission order
    entry_tile: np.ndarray
    keys: np.ndarray             # emission order, uint64
    sorted_keys: np.ndarray
    sorted_gauss: np.ndarray
    ranges: np.ndarray           # [n_tiles, 2]
    tiles: np.ndarray            # tiles that were blended
    images: dict = field(default_factory=dict)   # mode -> [3, H, W] (NaN outside blended tiles)
    T_final: np.ndarray | None = None            # primary mode, [H, W]
    n_proc: np.ndarray | None = None             # primary mode, [H, W]
    n_blend: np.ndarray | None = None            # primary mode, [H, W]
    c_max: np.ndarray | None = None
    slack: np.ndarray | None = None
    flagged: np.ndarray | None = None
    mode_slack: np.ndarray | None = None

    @property
    def image(self) -> np.ndarray:
        return self.images[self.modes[0]]

    key64: bool = False          # the fast path keyed like the plain one (ablation)

    @property
    def key_shift(self) -> int:
        return 32 if (self.path == "plain" or self.key64) else self.plan.b_d


_SHARED: dict = {}


def _tile_pixels(t: int, plan: FramePlan):
    tx, ty = t % plan.tiles_x, t // plan.tiles_x
    xs = np.arange(tx * TILE, min((tx + 1) * TILE, plan.width))
    ys = np.arange(ty * TILE, min((ty + 1) * TILE, plan.height))
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    return X.ravel(), Y.ravel()


def _blend_tiles(tiles):
    s = _SHARED
    out = []
    for t in tiles:
        a, b = s["ranges"][t]
        X, Y = _tile_pixels(int(t), s["plan"])
        r = blend_tile(s["sorted_gauss"][a:b], X.astype(np.float64), Y.astype(np.float64),
                       s["u"], s["v"], s["conic"], s["opa"], s["color"], modes=s["modes"],
                       bg=s["bg"], margins=s["margins"], margin_frame=s["margin_frame"])
        out.append((int(t), X, Y, r))
    return out


def render(arrays: dict, cam, path: str = "plain", modes=None, tiles=None, margins=None,
           workers: int = 1, blend: bool = True, alpha_extent: bool = True,
           key64: bool = False, exact_tiles: bool = False, margin_frame=None) -> OracleFrame:
    """Render one frame.  ``tiles`` restricts blending to a subset of tiles.

    For the fast path, ``alpha_extent=False`` keeps the 3-sigma tile extent
    and ``key64=True`` sorts on the plain path's (tile, float32 depth) key:
    the ablations of the opacity-culling step and of the 32-bit key.
    ``exact_tiles=True`` adds the exact ellipse-tile test to the alpha-ellipse
    extent (see ``tiles.ellipse_meets_tile``).  ``margin_frame`` is passed to
    ``blend.blend_tile``: decision bookkeeping only.
    """
    if path not in ("plain", "fast"):
        raise ValueError(path)
    fast = path == "fast"
    if modes is None:
        modes = ("fast-def", "fast-exact") if fast else ("plain",)
    plan = frame_plan(cam.width, cam.height)
    proj = project(arrays, cam, plan, fast, alpha_extent)
    eg, et = duplicate(proj.rect, proj.visible, plan)
    if exact_tiles:
        if not (fast and alpha_extent):
            raise ValueError("the exact ellipse-tile test refines the fast path's alpha-ellipse extent")
        eg, et = exact_tile_filter(eg, et, proj.rect, proj.u, proj.v, proj.cov, proj.det,
                                   arrays["log_opacity"], plan)
    d = proj.d[eg]
    key32 = fast and not key64
    keys = fast_keys(et, d, cam.z_near, cam.z_far, plan) if key32 else plain_keys(et, d)
    sk, sg = sort_entries(keys, eg)
    shift = plan.b_d if key32 else 32
    ranges = tile_ranges(sk, shift, plan.n_tiles)
    if tiles is None:
        tiles = np.arange(plan.n_tiles)
    tiles = np.asarray(tiles, np.int64)
    frame = OracleFrame(plan=plan, path=path, modes=tuple(modes), proj=proj, entry_gauss=eg,
                        entry_tile=et, keys=keys, sorted_keys=sk, sorted_gauss=sg, ranges=ranges,
                        tiles=tiles, key64=fast and key64)
    if not blend:
        return frame

    H, W = cam.height, cam.width
    for m in modes:
        frame.images[m] = np.full((3, H, W), np.nan)
    frame.T_final = np.full((H, W), np.nan)
    frame.n_proc = np.zeros((H, W), np.int64)
    frame.n_blend = np.zeros((H, W), np.int64)
    frame.c_max = np.zeros((H, W))
    frame.slack = np.zeros((H, W))
    frame.flagged = np.zeros((H, W), bool)
    frame.mode_slack = np.zeros((H, W))

    _SHARED.clear()
    _SHARED.update(plan=plan, ranges=ranges, sorted_gauss=sg, u=proj.u, v=proj.v, conic=proj.conic,
                   opa=arrays["log_opacity"] if fast else arrays["opacity"], color=proj.color,
                   modes=tuple(modes), bg=np.asarray(cam.bg, np.float64), margins=margins,
                   margin_frame=margin_frame)
    if workers > 1 and tiles.size > workers:
        chunks = np.array_split(tiles, workers * 4)
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_blend_tiles, chunks)
        results = [r for part in parts for r in part]
    else:
        results = _blend_tiles(tiles)
    for _, X, Y, r in results:
        for mi, m in enumerate(modes):
            frame.images[m][:, Y, X] = r.color[mi]
        frame.T_final[Y, X] = r.T[0]
        frame.n_proc[Y, X] = r.n_proc[0]
        frame.n_blend[Y, X] = r.n_blend[0]
        frame.c_max[Y, X] = r.c_max
        frame.slack[Y, X] = r.slack
        frame.flagged[Y, X] = r.flagged
        frame.mode_slack[Y, X] = r.mode_slack
    _SHARED.clear()
    return frame
