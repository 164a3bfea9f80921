"""The oracle's adjoint (reverse-mode derivative of the plain render) against
finite differences of the oracle's forward render, in float64 (CPU only).

Workload: 64 Gaussians at 64x64 (the finite-difference check of the
differentiation workload), loss L = sum(w * image) with seeded weights w.
Gradients are checked along seeded random directions within each parameter
group: means, log-scales, quaternions, opacity logits, SH DC and higher SH
terms, with the log-scale and logit chains (exp, sigmoid) applied by hand.
No decision (skip, stop, clamp, tile membership) may flip inside the finite
difference step; the test asserts that it does not.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import backward as OB

H = 64
W = 64


def raw_scene(seed=11, n=64):
    rng = np.random.Generator(np.random.PCG64(seed))
    return dict(
        means=rng.uniform(-0.8, 0.8, (n, 3)),
        log_scales=rng.normal(-2.4, 0.4, (n, 3)),
        quats=rng.normal(0.0, 1.0, (n, 4)),
        logits=rng.normal(0.5, 1.5, n),
        sh=np.concatenate([rng.normal(0.0, 0.5, (n, 1, 3)), rng.normal(0.0, 0.15, (n, 15, 3))], axis=1),
    )


def activate(raw):
    return dict(means=raw["means"], scales=np.exp(raw["log_scales"]), quats=raw["quats"],
                opacity=1.0 / (1.0 + np.exp(-raw["logits"])), sh=raw["sh"])


def camera(bg=(0.1, 0.3, 0.2)):
    cam = wl.config_camera("small", width=W, height=H)
    cam.bg = np.asarray(bg, np.float32)
    return cam


def loss_and_frame(raw, cam, w):
    fr = oracle.render(activate(raw), cam, "plain")
    return float(np.sum(w * fr.image)), fr


def raw_gradients(raw, cam, w):
    arr = activate(raw)
    adj = OB.render_adjoint(arr, cam, w)
    g = adj.params
    o = arr["opacity"]
    return dict(means=g.means, log_scales=g.scales * arr["scales"], quats=g.quats,
                logits=g.opacity * o * (1.0 - o), sh=g.sh), adj


GROUPS = {
    "means": ("means", None),
    "log_scales": ("log_scales", None),
    "quats": ("quats", None),
    "logits": ("logits", None),
    "sh_dc": ("sh", slice(0, 1)),
    "sh_rest": ("sh", slice(1, 16)),
}


@pytest.fixture(scope="module")
def setup():
    raw = raw_scene()
    cam = camera()
    rng = np.random.Generator(np.random.PCG64(5))
    w = rng.normal(0.0, 1.0, (3, H, W))
    grads, adj = raw_gradients(raw, cam, w)
    return raw, cam, w, grads, adj


def test_fixture_has_blending_overlap_and_no_near_decisions(setup):
    raw, cam, w, grads, adj = setup
    fr = oracle.render(activate(raw), cam, "plain")
    assert fr.proj.visible.sum() >= 48
    assert (fr.n_blend >= 3).mean() > 0.2, "too little overlap to exercise the blending adjoint"
    assert not adj.pixel_flagged.any() and not adj.flagged.any()
    assert np.isfinite(fr.image).all()


@pytest.mark.parametrize("group", list(GROUPS))
@pytest.mark.parametrize("k", [0, 1])
def test_directional_derivative_matches_finite_differences(setup, group, k):
    raw, cam, w, grads, _ = setup
    key, sl = GROUPS[group]
    rng = np.random.Generator(np.random.PCG64(100 + 7 * k + len(group)))
    direction = np.zeros_like(raw[key])
    if sl is None:
        direction[...] = rng.normal(0.0, 1.0, raw[key].shape)
    else:
        direction[:, sl] = rng.normal(0.0, 1.0, direction[:, sl].shape)
    h = 1e-6
    plus = {**raw, key: raw[key] + h * direction}
    minus = {**raw, key: raw[key] - h * direction}
    Lp, fp = loss_and_frame(plus, cam, w)
    Lm, fm = loss_and_frame(minus, cam, w)
    _, f0 = loss_and_frame(raw, cam, w)
    for f in (fp, fm):       # the same discrete decisions on both sides
        assert np.array_equal(f.proj.rect, f0.proj.rect)
        assert np.array_equal(f.sorted_gauss, f0.sorted_gauss)
        assert np.array_equal(f.n_proc, f0.n_proc) and np.array_equal(f.n_blend, f0.n_blend)
    fd = (Lp - Lm) / (2.0 * h)
    an = float(np.sum(grads[key] * direction))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (group, fd, an)


def test_single_isotropic_gaussian_closed_form():
    """One isotropic Gaussian on the optical axis: at the pixel under its mean,
    image = c o + (1 - o) bg with c = 0.5 + sum_k Y_k(dir) k_k, so dI/do = c - bg
    and dI/dk_k = o Y_k(dir) per channel; dir = (0, 0, 1), where only the m = 0
    functions are nonzero: Y_0 = 1/(2 sqrt(pi)), Y_2 = sqrt(3/(4 pi)),
    Y_6 = sqrt(5/pi)/2, Y_12 = sqrt(7/pi)/2.  Its 2D mean sits on the pixel, where
    the gradients of u and v vanish by symmetry."""
    cam = wl.look_at_camera((0, 0, -3.0), (0, 0, 0), (0, 1, 0), 60.0, 33, 33, 1.0, 5.0,
                            bg=(0.25, 0.5, 0.125))
    o, kdc = 0.6, np.array([0.3, -0.2, 0.1])
    arr = dict(means=np.zeros((1, 3)), scales=np.full((1, 3), 0.05), quats=np.array([[1.0, 0, 0, 0]]),
               opacity=np.array([o]), sh=np.zeros((1, 16, 3)))
    arr["sh"][0, 0] = kdc
    y00 = 0.5 / math.sqrt(math.pi)
    c = 0.5 + y00 * kdc
    w = np.zeros((3, 33, 33))
    w[:, 16, 16] = 1.0               # pixel (16, 16) is the centre: cx = cy = 16
    adj = OB.render_adjoint(arr, cam, w)
    bg = np.asarray(cam.bg, np.float64)
    assert math.isclose(adj.params.opacity[0], float(np.sum(c - bg)), rel_tol=1e-12)
    yz = np.zeros(16)
    yz[0], yz[2], yz[6], yz[12] = y00, math.sqrt(3 / (4 * math.pi)), math.sqrt(5 / math.pi) / 2, \
        math.sqrt(7 / math.pi) / 2
    assert np.allclose(adj.params.sh[0], o * yz[:, None], rtol=1e-12, atol=1e-15)
    assert abs(adj.screen[0, 0]) < 1e-12 and abs(adj.screen[0, 1]) < 1e-12


def test_clamped_alpha_has_no_opacity_gradient():
    cam = wl.look_at_camera((0, 0, -3.0), (0, 0, 0), (0, 1, 0), 60.0, 33, 33, 1.0, 5.0)
    arr = dict(means=np.zeros((1, 3)), scales=np.full((1, 3), 0.2), quats=np.array([[1.0, 0, 0, 0]]),
               opacity=np.array([0.999]), sh=np.zeros((1, 16, 3)))
    w = np.zeros((3, 33, 33))
    w[:, 16, 16] = 1.0               # alpha = min(0.99, 0.999) there
    adj = OB.render_adjoint(arr, cam, w)
    assert adj.params.opacity[0] == 0.0
