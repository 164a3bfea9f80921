"""Planted mistakes in the oracle's adjoint must fail its finite-difference pin
(CPU only).  Each case patches one helper of the adjoint with a plausible slip
and checks that some parameter group's directional derivative now disagrees
with finite differences of the (unpatched) forward render."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import backward as OB
from test_oracle_backward import GROUPS, activate, camera, loss_and_frame, raw_scene

H = W = 64


def worst_deviation(raw, cam, w):
    arr = activate(raw)
    g = OB.render_adjoint(arr, cam, w).params
    o = arr["opacity"]
    grads = dict(means=g.means, log_scales=g.scales * arr["scales"], quats=g.quats,
                 logits=g.opacity * o * (1.0 - o), sh=g.sh)
    worst = 0.0
    rng = np.random.Generator(np.random.PCG64(77))
    for group, (key, sl) in GROUPS.items():
        d = np.zeros_like(raw[key])
        if sl is None:
            d[...] = rng.normal(0.0, 1.0, d.shape)
        else:
            d[:, sl] = rng.normal(0.0, 1.0, d[:, sl].shape)
        h = 1e-6
        Lp, _ = loss_and_frame({**raw, key: raw[key] + h * d}, cam, w)
        Lm, _ = loss_and_frame({**raw, key: raw[key] - h * d}, cam, w)
        fd = (Lp - Lm) / (2 * h)
        an = float(np.sum(grads[key] * d))
        worst = max(worst, abs(fd - an) / max(1.0, abs(fd)))
    return worst


def _no_view_direction(mp):
    mp.setattr(OB, "sh_basis_jacobian", lambda dirs: np.zeros((dirs.shape[0], 16, 3)))


def _transposed_rotation_jacobian(mp):
    orig = OB.rotation_jacobian
    mp.setattr(OB, "rotation_jacobian", lambda q: orig(q).transpose(0, 2, 1, 3))


def _camera_centre_sign(mp):
    orig = OB.camera_center
    mp.setattr(OB, "camera_center", lambda cam: -orig(cam))


def _no_jacobian_clamp(mp):
    mp.setattr(OB, "J_CLAMP", 0.5)


def _alpha_clamp_ignored(mp):
    mp.setattr(OB, "ALPHA_MAX", 1e9)


MUTATIONS = [_no_view_direction, _transposed_rotation_jacobian, _camera_centre_sign, _no_jacobian_clamp,
             _alpha_clamp_ignored]


@pytest.fixture(scope="module")
def base():
    raw = raw_scene()
    raw["logits"] = raw["logits"] + 2.5        # many opaque Gaussians: clamped alphas occur
    cam = camera()
    w = np.random.Generator(np.random.PCG64(5)).normal(0.0, 1.0, (3, H, W))
    return raw, cam, w


def test_unpatched_adjoint_passes(base):
    assert worst_deviation(*base) < 1e-6


@pytest.mark.parametrize("mutate", MUTATIONS, ids=lambda f: f.__name__)
def test_planted_mistake_is_caught(base, mutate, monkeypatch):
    mutate(monkeypatch)
    assert worst_deviation(*base) > 1e-3
