"""Duplication, sorting keys, depth sort and tile ranges.

Sec. III-B: every visible Gaussian is duplicated once per tile its extent
covers; each duplicate carries a (tile, depth) key and the Gaussian index.
Sec. III-C / IV-A: the entries are radix-sorted by key, so that entries are
grouped by tile and ordered front to back by depth inside a tile.

* plain key (the 3DGS baseline, Sec. IV-A): 64 bits, tile index in the upper
  32 bits, the bit pattern of the FP32 depth in the lower 32 bits (depth > 0,
  so the float bits order like the values);
* fast key (Eq. depth_quant): 32 bits, tile index in the upper b_t bits and
  q_d = clamp(floor((d - z_near) / (z_far - z_near) * (2^b_d - 1)), 0,
  2^b_d - 1) in the lower b_d bits, evaluated in float64 in that order.

Readings: entries of one Gaussian are emitted in row-major tile order and the
Gaussians in index order; the sort orders by (key, Gaussian index), so equal
keys keep index order.  "Front-to-back" is the order the blending needs
(Eq. alpha_computation); Sec. II-A's "back-to-front" is read as a slip.
Tile ranges are the maximal runs of equal tile index in the sorted list.
"""
from __future__ import annotations

import numpy as np

from .plan import FramePlan
from .project import LN255


def duplicate(rect: np.ndarray, visible: np.ndarray, plan: FramePlan):
    """Per-entry (Gaussian index, tile index), in emission order."""
    idx = np.nonzero(visible)[0]
    x0, x1, y0, y1 = (rect[idx, k] for k in range(4))
    w = x1 - x0 + 1
    count = w * (y1 - y0 + 1)
    starts = np.concatenate([[0], np.cumsum(count)[:-1]])
    g = np.repeat(np.arange(idx.size), count)
    local = np.arange(int(count.sum())) - starts[g]
    tx = x0[g] + local % w[g]
    ty = y0[g] + local // w[g]
    return idx[g].astype(np.int64), (ty * plan.tiles_x + tx).astype(np.int64)


# The exact ellipse-tile test (an extension of the fast path's culling step,
# Sec. IV-A: the tile-precise half of the Speedy-Splat culling).  A tile is
# kept iff the box of its pixel centres [16 tx, 16 tx + 15] x [16 ty, 16 ty + 15]
# holds a point of the ellipse q(p) <= tau, where q(p) = (c11 dx^2 - 2 c01 dx dy
# + c00 dy^2) / det for p - (u, v) = (dx, dy) and tau = 2 (ln 255 + ln o): the
# pixels outside that ellipse have alpha < 1/255.  Only rectangles of at most
# EXACT_TILE_MAX_AREA tiles are filtered; larger ones keep every tile.
#
# Reading (the paper names the culling strategy but not its arithmetic): q is
# convex, so the box meets the ellipse iff it holds the mean or one of its four
# edges does.  On the line x = X the least q is dx^2 / c00 at dy = c01 dx / c00;
# if that dy lies off the edge, the least q on the edge is at the nearer
# corner.  Every comparison is multiplied through by c00, c11 or det (> 0), in
# float64, evaluated left to right as written (the key-defining arithmetic).
EXACT_TILE_MAX_AREA = 64


def ellipse_meets_tile(u, v, c00, c01, c11, det, tau, tx, ty) -> np.ndarray:
    """Elementwise: does the alpha >= 1/255 ellipse of a Gaussian meet tile (tx, ty)?"""
    X0 = 16.0 * np.asarray(tx, np.float64)
    Y0 = 16.0 * np.asarray(ty, np.float64)
    X1 = X0 + 15.0
    Y1 = Y0 + 15.0
    keep = (u >= X0) & (u <= X1) & (v >= Y0) & (v <= Y1)
    rhs = tau * det
    for Xe in (X0, X1):
        dx = Xe - u
        t = c01 * dx
        lo = (Y0 - v) * c00
        hi = (Y1 - v) * c00
        inner = (t >= lo) & (t <= hi)
        dy = np.where(t < lo, Y0 - v, Y1 - v)
        near = c11 * dx * dx - 2.0 * c01 * dx * dy + c00 * dy * dy <= rhs
        keep |= np.where(inner, dx * dx <= tau * c00, near)
    for Ye in (Y0, Y1):
        dy = Ye - v
        t = c01 * dy
        lo = (X0 - u) * c11
        hi = (X1 - u) * c11
        inner = (t >= lo) & (t <= hi)
        dx = np.where(t < lo, X0 - u, X1 - u)
        near = c11 * dx * dx - 2.0 * c01 * dx * dy + c00 * dy * dy <= rhs
        keep |= np.where(inner, dy * dy <= tau * c11, near)
    return keep


def exact_tile_filter(entry_gauss, entry_tile, rect, u, v, cov, det, log_opacity, plan: FramePlan):
    """Entries (in emission order) that the exact ellipse-tile test keeps."""
    x0, x1, y0, y1 = (rect[entry_gauss, k] for k in range(4))
    area = (x1 - x0 + 1) * (y1 - y0 + 1)
    tx = entry_tile % plan.tiles_x
    ty = entry_tile // plan.tiles_x
    g = entry_gauss
    tau = 2.0 * (LN255 + log_opacity[g])
    meets = ellipse_meets_tile(u[g], v[g], cov[g, 0], cov[g, 1], cov[g, 2], det[g], tau, tx, ty)
    keep = (area > EXACT_TILE_MAX_AREA) | meets
    return entry_gauss[keep], entry_tile[keep]


def plain_keys(tile: np.ndarray, depth_of_entry: np.ndarray) -> np.ndarray:
    """64-bit key: tile << 32 | bits(fp32(d))."""
    bits = depth_of_entry.astype(np.float32).view(np.uint32).astype(np.uint64)
    return (tile.astype(np.uint64) << np.uint64(32)) | bits


def quantize_depth(d: np.ndarray, z_near: float, z_far: float, b_d: int) -> np.ndarray:
    """Eq. depth_quant in float64, evaluated as written (divide, then scale)."""
    levels = float((1 << b_d) - 1)
    q = np.floor((d - z_near) / (z_far - z_near) * levels)
    return np.clip(q, 0.0, levels).astype(np.uint64)


def fast_keys(tile: np.ndarray, depth_of_entry: np.ndarray, z_near: float, z_far: float,
              plan: FramePlan) -> np.ndarray:
    """32-bit key: tile << b_d | q_d (returned as uint64 holding 32 significant bits)."""
    q = quantize_depth(depth_of_entry, z_near, z_far, plan.b_d)
    return (tile.astype(np.uint64) << np.uint64(plan.b_d)) | q


def sort_entries(keys: np.ndarray, gauss: np.ndarray):
    """Entries ordered by (key, Gaussian index); returns (sorted keys, sorted indices)."""
    order = np.lexsort((gauss, keys))
    return keys[order], gauss[order]


def tile_ranges(sorted_keys: np.ndarray, shift: int, n_tiles: int) -> np.ndarray:
    """[n_tiles, 2] start/end of each tile's run in the sorted list (empty: 0, 0)."""
    tiles = (sorted_keys >> np.uint64(shift)).astype(np.int64)
    t = np.arange(n_tiles)
    start = np.searchsorted(tiles, t, side="left")
    end = np.searchsorted(tiles, t, side="right")
    empty = start == end
    start[empty] = 0
    end[empty] = 0
    return np.stack([start, end], axis=1)
