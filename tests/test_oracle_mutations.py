"""Planted mistakes in the oracle must make at least one pin fail (CPU only).

Each case patches one oracle function or constant with a plausible slip (a
transposed operand, a wrong sign, a dropped term, an off-by-one) and checks
that the independent pin named beside it now reports a large deviation.
"""
from __future__ import annotations

import importlib

import numpy as np
import pytest

import oracle_checks as oc

PROJECT = importlib.import_module("oracle.project")
RENDER = importlib.import_module("oracle.render")
BLEND = importlib.import_module("oracle.blend")
FASTEXP = importlib.import_module("oracle.fastexp")
TILES = importlib.import_module("oracle.tiles")

ANISO = dict(quat=(0.8, 0.3, -0.4, 0.33), scales=(0.09, 0.03, 0.05))


def _transposed_rotation(mp):
    orig = PROJECT.quat_to_rotation
    mp.setattr(PROJECT, "quat_to_rotation", lambda q: orig(q).transpose(0, 2, 1))
    return lambda: oc.check_single_gaussian(**ANISO)


def _conic_sign(mp):
    orig = RENDER.project

    def wrong(*a, **k):
        pr = orig(*a, **k)
        pr.conic[:, 1] *= -1.0
        return pr
    mp.setattr(RENDER, "project", wrong)
    return lambda: oc.check_single_gaussian(**ANISO)


def _no_dilation(mp):
    mp.setattr(PROJECT, "DILATION", 0.0)
    return lambda: oc.check_single_gaussian()


def _no_jacobian_clamp(mp):
    mp.setattr(PROJECT, "J_CLAMP", 1e9)
    return oc.check_off_axis_jacobian


def _back_to_front(mp):
    def wrong(keys, gauss):
        order = np.lexsort((gauss, keys))[::-1]
        return keys[order], gauss[order]
    mp.setattr(RENDER, "sort_entries", wrong)
    return oc.check_depth_order_and_stop


def _no_stop(mp):
    mp.setattr(BLEND, "T_MIN", 0.0)
    return oc.check_depth_order_and_stop


def _no_clamp(mp):
    mp.setattr(BLEND, "ALPHA_MAX", 1.0)
    return oc.check_depth_order_and_stop


def _no_skip(mp):
    mp.setattr(BLEND, "ALPHA_MIN", 0.0)
    return lambda: oc.check_single_gaussian()


def _sh_sign(mp):
    orig = PROJECT.sh_basis

    def wrong(d):
        Y = orig(d)
        Y[:, 1] *= -1.0
        return Y
    mp.setattr(PROJECT, "sh_basis", wrong)
    return oc.check_sh_basis


def _sigma_sign(mp):
    mp.setattr(FASTEXP, "SIGMA", -FASTEXP.SIGMA)
    return oc.check_fast_exp_envelope


def _short_rect(mp):
    orig = PROJECT.tile_rect

    def wrong(*a, **k):
        r = orig(*a, **k)
        r[:, 1] -= 1.0
        return r
    mp.setattr(PROJECT, "tile_rect", wrong)
    return lambda: oc.check_single_gaussian()


def _tile_index_transposed(mp):
    orig = TILES.duplicate

    def wrong(rect, visible, plan):
        g, t = orig(rect, visible, plan)
        tx, ty = t % plan.tiles_x, t // plan.tiles_x
        return g, tx * plan.tiles_y + ty
    mp.setattr(RENDER, "duplicate", wrong)
    return lambda: oc.check_brute_force("plain")


def _exact_tile_off_diagonal_sign(mp):
    orig = TILES.ellipse_meets_tile
    mp.setattr(TILES, "ellipse_meets_tile",
               lambda u, v, c00, c01, c11, det, tau, tx, ty: orig(u, v, c00, -c01, c11, det, tau, tx, ty))
    mp.setattr(oc.oracle, "ellipse_meets_tile", TILES.ellipse_meets_tile)
    return oc.check_exact_tile_test


def _exact_tile_swapped_axes(mp):
    orig = TILES.ellipse_meets_tile
    mp.setattr(TILES, "ellipse_meets_tile",
               lambda u, v, c00, c01, c11, det, tau, tx, ty: orig(u, v, c11, c01, c00, det, tau, tx, ty))
    mp.setattr(oc.oracle, "ellipse_meets_tile", TILES.ellipse_meets_tile)
    return oc.check_exact_tile_test


def _exact_tile_box_one_short(mp):
    orig = TILES.ellipse_meets_tile
    mp.setattr(TILES, "ellipse_meets_tile",
               lambda u, v, c00, c01, c11, det, tau, tx, ty: orig(u - 1.0, v - 1.0, c00, c01, c11, det, tau, tx, ty)
               & orig(u, v, c00, c01, c11, det, tau, tx, ty))
    mp.setattr(oc.oracle, "ellipse_meets_tile", TILES.ellipse_meets_tile)
    return oc.check_exact_tile_test


MUTATIONS = {
    "transposed rotation": _transposed_rotation,
    "conic off-diagonal sign": _conic_sign,
    "dropped 0.3 dilation": _no_dilation,
    "dropped Jacobian clamp": _no_jacobian_clamp,
    "back-to-front order": _back_to_front,
    "no early stop": _no_stop,
    "no 0.99 clamp": _no_clamp,
    "no 1/255 skip": _no_skip,
    "SH sign": _sh_sign,
    "sigma sign": _sigma_sign,
    "short tile rectangle": _short_rect,
    "transposed tile index": _tile_index_transposed,
    "exact tile test: off-diagonal sign": _exact_tile_off_diagonal_sign,
    "exact tile test: swapped axes": _exact_tile_swapped_axes,
    "exact tile test: box one pixel short": _exact_tile_box_one_short,
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_pin_catches_planted_mistake(name, monkeypatch):
    check = MUTATIONS[name](monkeypatch)
    try:
        dev = check()
    except (AssertionError, IndexError, ValueError):
        return                              # the check itself tripped on the mistake
    assert dev > 1e-4, f"{name}: pin deviation only {dev}"
