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
