"""Tile grid and the resolution-adaptive key bit split.

Sec. IV-A, "Resolution-Adaptive Sorting-Key Encoding": with N_t = T_x * T_y
tiles of 16x16 pixels, the tile index takes b_t = ceil(log2 N_t) bits in the
high part of a 32-bit key and the quantised depth the remaining b_d = 32 - b_t
low bits.  Reading (paper silent): for N_t = 1 the formula gives b_t = 0; we
keep at least one tile bit, b_t = max(1, ceil(log2 N_t)).
"""
from __future__ import annotations

from dataclasses import dataclass

TILE = 16


def key_bits(n_tiles: int) -> tuple[int, int]:
    """(b_t, b_d) for a grid of n_tiles tiles, in exact integer arithmetic."""
    if n_tiles < 1:
        raise ValueError("n_tiles must be positive")
    b_t = max(1, (n_tiles - 1).bit_length())   # ceil(log2 n) for n >= 1
    return b_t, 32 - b_t


@dataclass(frozen=True)
class FramePlan:
    width: int
    height: int
    tiles_x: int
    tiles_y: int
    n_tiles: int
    b_t: int
    b_d: int

    @property
    def depth_levels(self) -> int:
        return 1 << self.b_d

    @property
    def plain_key_bits(self) -> int:
        """Significant bits of the 64-bit (tile | float depth) key."""
        return 32 + self.b_t


def frame_plan(width: int, height: int) -> FramePlan:
    tx = -(-width // TILE)
    ty = -(-height // TILE)
    b_t, b_d = key_bits(tx * ty)
    return FramePlan(width, height, tx, ty, tx * ty, b_t, b_d)
