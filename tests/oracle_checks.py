"""Independent checks that pin the FP64 oracle to things other than itself.

Each check returns the largest deviation it finds (0 when exact), so that the
pin tests can assert on it and the mutation tests can show that a planted
mistake in the oracle makes the same check fail.  The expected values come
from closed forms, library routines (scipy's spherical harmonics and
rotations, numpy's linear algebra) or brute force written here, never from
the oracle's own intermediate results.
"""
from __future__ import annotations

import importlib
import math
from fractions import Fraction

import numpy as np

import oracle
import workloads as wl

# the package re-exports functions under its submodules' names; reach the modules directly
PROJECT = importlib.import_module("oracle.project")

Y00 = 0.5 / math.sqrt(math.pi)


def tiny_scene(means, scales, quats, opacity, colors):
    """float32 scene whose SH holds only the DC term that yields ``colors``."""
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = means.shape[0]
    sh = np.zeros((n, 16, 3))
    sh[:, 0, :] = (np.asarray(colors, np.float64).reshape(n, 3) - 0.5) / Y00
    return wl.Scene(means=means.astype(np.float32),
                    scales=np.asarray(scales, np.float64).reshape(n, 3).astype(np.float32),
                    quats=np.asarray(quats, np.float64).reshape(n, 4).astype(np.float32),
                    opacity=np.asarray(opacity, np.float64).reshape(n).astype(np.float32),
                    sh=sh.astype(np.float32))


def axis_camera(D=3.0, W=64, H=48, fovx=60.0, reach=1.5):
    """Camera on the -z axis looking at the origin (camera rotation diag(-1, -1, 1))."""
    return wl.look_at_camera((0.0, 0.0, -D), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), fovx, W, H,
                             max(0.2, D - reach), D + reach)


def scene_colors(scene):
    """RGB of a DC-only scene, as the SH definition gives it."""
    return np.maximum(0.0, 0.5 + Y00 * scene.sh[:, 0, :].astype(np.float64))


def pixel_grid(cam):
    j, i = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    return i.astype(np.float64), j.astype(np.float64)


def closed_form_single(scene, cam):
    """Image of one Gaussian at the origin seen on axis, from the EWA definition.

    Sigma' = J R_w Sigma R_w^T J^T + 0.3 I with J = diag(fx/D, fy/D) (on axis),
    Sigma from scipy's rotation of the quaternion; alpha = min(0.99, o exp(-q/2))
    with q the Mahalanobis form of Sigma'^-1 (numpy inverse), kept where
    alpha >= 1/255.  Opacity must be small enough that every such pixel lies
    inside the 3-sigma extent, so the tile rule does not enter.
    """
    from scipy.spatial.transform import Rotation

    q = scene.quats[0].astype(np.float64)
    Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    s2 = np.diag(scene.scales[0].astype(np.float64) ** 2)
    Sigma = Rm @ s2 @ Rm.T
    D = float(cam.t[2])
    J = np.array([[cam.fx / D, 0.0, 0.0], [0.0, cam.fy / D, 0.0]])
    cov2 = J @ cam.R @ Sigma @ cam.R.T @ J.T + 0.3 * np.eye(2)
    inv = np.linalg.inv(cov2)
    X, Y = pixel_grid(cam)
    dx, dy = X - cam.cx, Y - cam.cy
    maha = inv[0, 0] * dx * dx + 2 * inv[0, 1] * dx * dy + inv[1, 1] * dy * dy
    alpha = np.minimum(0.99, float(scene.opacity[0]) * np.exp(-0.5 * maha))
    alpha = np.where(alpha >= 1.0 / 255.0, alpha, 0.0)
    c = scene_colors(scene)[0]
    return c[:, None, None] * alpha[None]


def check_single_gaussian(quat=(1.0, 0.0, 0.0, 0.0), scales=(0.05, 0.05, 0.05), opacity=0.3,
                          color=(0.8, 0.4, 0.2), path="plain"):
    sc = tiny_scene([0, 0, 0], scales, quat, opacity, color)
    cam = axis_camera()
    arr = oracle.prepare_plain(sc)
    if path == "fast":
        arr = dict(arr)
        arr["log_opacity"] = np.log(arr.pop("opacity"))
        fr = oracle.render(arr, cam, "fast", modes=("fast-exact",))
    else:
        fr = oracle.render(arr, cam, "plain")
    return float(np.max(np.abs(fr.image - closed_form_single(sc, cam))))


def check_off_axis_jacobian(x0=0.6, clamp_x0=3.0, s=0.05):
    """Sigma'_00, Sigma'_11, u of an isotropic Gaussian at (x0, 0, 0), on and past the clamp.

    With camera rotation diag(-1,-1,1) the Gaussian sits at t = (-x0, 0, D); the
    EWA Jacobian of the pinhole is J = [[fx/D, 0, -fx xc/D^2], [0, fy/D, 0]] with
    xc = clamp(t_x/D, +-1.3 tan(fovx/2)) D, and Sigma' = s^2 J J^T + 0.3 I.
    """
    cam = axis_camera(W=256, H=256)
    D = float(cam.t[2])
    worst = 0.0
    for x in (x0, clamp_x0):
        sc = tiny_scene([x, 0, 0], [s, s, s], [1, 0, 0, 0], 0.5, [0.5, 0.5, 0.5])
        arr = oracle.prepare_plain(sc)
        plan = oracle.frame_plan(cam.width, cam.height)
        pr = oracle.project(arr, cam, plan, fast=False)
        xs = float(sc.means[0, 0])
        ss = float(sc.scales[0, 0])
        tx = -xs
        lim = 1.3 * cam.tan_half_fovx
        xc = max(-lim, min(lim, tx / D)) * D
        c00 = ss * ss * (cam.fx ** 2 / D ** 2 + cam.fx ** 2 * xc ** 2 / D ** 4) + 0.3
        c11 = ss * ss * cam.fy ** 2 / D ** 2 + 0.3
        u = cam.fx * tx / D + cam.cx
        rel = max(abs(pr.cov[0, 0] - c00) / c00, abs(pr.cov[0, 2] - c11) / c11,
                  abs(pr.cov[0, 1]), abs(pr.u[0] - u) / abs(u), abs(pr.d[0] - D) / D)
        worst = max(worst, rel)
    return worst


def check_depth_order_and_stop():
    """Coincident Gaussians at the image centre, listed far-to-near.

    Two Gaussians: C = c1 a1 + c2 a2 (1 - a1) with 1 the nearer one.
    Four Gaussians of centre alpha 0.95: T after k is 0.05^k, the fourth would
    take T to 6.25e-6 < 1e-4 and is not blended.
    Returns the largest error at the centre pixel.
    """
    W = H = 33                      # odd: the centre pixel sits on the optical axis
    cam = axis_camera(W=W, H=H)
    D = float(cam.t[2])
    worst = 0.0
    # two Gaussians, far one first in index order
    sc = tiny_scene([[0, 0, 0.5], [0, 0, -0.5]], [[0.05] * 3] * 2, [[1, 0, 0, 0]] * 2, [0.7, 0.6],
                    [[0.9, 0.1, 0.1], [0.1, 0.2, 0.9]])
    fr = oracle.render(oracle.prepare_plain(sc), cam, "plain")
    a = [float(sc.opacity[k]) for k in range(2)]        # exp(0) at the centre
    c = scene_colors(sc)
    expect = c[1] * a[1] + c[0] * a[0] * (1 - a[1])
    worst = max(worst, float(np.max(np.abs(fr.image[:, H // 2, W // 2] - expect))))
    # four Gaussians, stop before the fourth
    z = [0.3, 0.1, -0.1, -0.3]
    cols = [[0.9, 0.0, 0.0], [0.0, 0.9, 0.0], [0.0, 0.0, 0.9], [0.9, 0.9, 0.9]]
    sc = tiny_scene([[0, 0, zz] for zz in z], [[0.05] * 3] * 4, [[1, 0, 0, 0]] * 4, [0.95] * 4, cols)
    fr = oracle.render(oracle.prepare_plain(sc), cam, "plain")
    a = float(sc.opacity[0])
    c = scene_colors(sc)
    near_first = [3, 2, 1]
    expect = sum(c[g] * a * (1 - a) ** k for k, g in enumerate(near_first))
    worst = max(worst, float(np.max(np.abs(fr.image[:, H // 2, W // 2] - expect))))
    worst = max(worst, abs(float(fr.T_final[H // 2, W // 2]) - (1 - a) ** 3))
    # one opaque Gaussian: the centre alpha is clamped to 0.99 (Eq. opacity_clamped)
    sc = tiny_scene([0, 0, 0], [0.05] * 3, [1, 0, 0, 0], 1.0, [0.6, 0.7, 0.8])
    fr = oracle.render(oracle.prepare_plain(sc), cam, "plain")
    expect = scene_colors(sc)[0] * 0.99
    worst = max(worst, float(np.max(np.abs(fr.image[:, H // 2, W // 2] - expect))))
    return worst


def check_sh_basis(n=2000, seed=0):
    """Real SH basis against scipy's complex SH (Condon-Shortley phase).

    Our real basis is sqrt(2) Re Y_l^m for m > 0, sqrt(2) Im Y_l^|m| for m < 0
    and Y_l^0 for m = 0, at index l*l + l + m.
    """
    from scipy.special import sph_harm_y

    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    ref = np.empty((n, 16))
    for l in range(4):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                val = math.sqrt(2) * Y.real
            elif m < 0:
                val = math.sqrt(2) * Y.imag
            else:
                val = Y.real
            ref[:, l * l + l + m] = val
    return float(np.max(np.abs(PROJECT.sh_basis(d) - ref)))


def check_rotation(n=2000, seed=0):
    """Rotation of (unnormalised) quaternions against scipy."""
    from scipy.spatial.transform import Rotation

    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4)) * rng.uniform(0.1, 10, size=(n, 1))
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    return float(np.max(np.abs(PROJECT.quat_to_rotation(q) - ref)))


def check_fast_exp_envelope(sigma_expected=0.045677):
    """Dense relative error of exp^ on [-ln 255, 0] against the closed-form envelope."""
    P = np.linspace(-math.log(255.0), 0.0, 400001)
    err = oracle.fast_exp_rel_error(P)
    two = 2.0 ** (-sigma_expected)
    f_star = 1.0 / math.log(2.0) - 1.0
    lo = two - 1.0
    hi = two * (1.0 + f_star) * 2.0 ** (-f_star) - 1.0
    # measured extremes must reach the envelope (within floor/grid effects) and stay inside
    return max(abs(err.min() - lo), abs(err.max() - hi),
               max(0.0, err.max() - hi - 2e-7), max(0.0, lo - err.min() - 2e-7))


def fp16_round_exact(x: float) -> float:
    """Round a double to binary16, nearest-even, with exact rational arithmetic."""
    if x == 0:
        return 0.0
    sign = -1.0 if x < 0 else 1.0
    fx = Fraction(abs(x))
    # binary16: 10 fraction bits, exponent range [-14, 15], subnormal spacing 2^-24
    e = math.floor(math.log2(abs(x)))
    while Fraction(2) ** e > fx:
        e -= 1
    while Fraction(2) ** (e + 1) <= fx:
        e += 1
    e = max(e, -14)
    ulp = Fraction(2) ** (e - 10)
    q, r = divmod(fx, ulp)
    if r * 2 > ulp or (r * 2 == ulp and q % 2 == 1):
        q += 1
    val = q * ulp
    if val > 65504:
        return sign * math.inf
    return sign * float(val)


def brute_force_image(arrays, cam, path, mode, key64=False, alpha_extent=True):
    """Per-pixel reference: every visible Gaussian whose tile rectangle holds the
    pixel's tile, ordered by (depth key, index), blended with a scalar loop.

    No duplication, sort or tile ranges; the projection is the oracle's.
    Also asserts the blending invariants along the way.  ``key64`` orders the
    fast path by float32 depth; ``alpha_extent`` selects its tile extent.
    """
    fast = path == "fast"
    plan = oracle.frame_plan(cam.width, cam.height)
    pr = oracle.project(arrays, cam, plan, fast, alpha_extent)
    vis = np.nonzero(pr.visible)[0]
    if fast and key64:
        dk = [int(np.float32(pr.d[g]).view(np.uint32)) for g in vis]
        opa = arrays["log_opacity"]
    elif fast:
        lv = (1 << plan.b_d) - 1
        dk = [min(max(math.floor((pr.d[g] - cam.z_near) / (cam.z_far - cam.z_near) * lv), 0), lv)
              for g in vis]
        opa = arrays["log_opacity"]
    else:
        dk = [int(np.float32(pr.d[g]).view(np.uint32)) for g in vis]
        opa = arrays["opacity"]
    order = [g for _, g in sorted(zip(dk, vis))]
    img = np.zeros((3, cam.height, cam.width))
    ln255 = math.log(255.0)
    for j in range(cam.height):
        for i in range(cam.width):
            tx, ty = i // 16, j // 16
            T = 1.0
            C = [0.0, 0.0, 0.0]
            cmax = 0.0
            for g in order:
                x0, x1, y0, y1 = pr.rect[g]
                if not (x0 <= tx <= x1 and y0 <= ty <= y1):
                    continue
                dx = i - pr.u[g]
                dy = j - pr.v[g]
                A, B, Cc = pr.conic[g]
                p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
                if fast:
                    P = p + opa[g]
                    if P < -ln255:
                        continue
                    assert P <= opa[g] + 1e-12
                    e = math.exp(P) if mode == "fast-exact" else float(oracle.fast_exp(P))
                    a = min(0.99, e)
                else:
                    a = min(0.99, opa[g] * math.exp(p))
                    if a < 1.0 / 255.0:
                        continue
                Tn = T * (1.0 - a)
                if Tn < 1e-4:
                    break
                cg = pr.color[g]
                for k in range(3):
                    C[k] += a * T * cg[k]
                cmax = max(cmax, float(np.max(cg)))
                assert 0.0 <= Tn <= T <= 1.0
                T = Tn
            for k in range(3):
                assert -1e-12 <= C[k] <= cmax * (1.0 - T) + 1e-12
                img[k, j, i] = C[k] + T * float(cam.bg[k])
    return img


def check_brute_force(path="plain", seed=5, n=40, W=45, H=37, key64=False, alpha_extent=True):
    sc = wl.make_scene(n, 1.0, -2.5, 0.4, seed)
    cam = wl.look_at_camera((0.0, 0.0, -3.0), (0, 0, 0), (0, 1, 0), 60.0, W, H, 1.268, 4.732)
    if path == "fast":
        arr = oracle.prepare_fast(oracle.quantize_scene(sc))
        mode = "fast-def"
        fr = oracle.render(arr, cam, "fast", modes=(mode,), key64=key64, alpha_extent=alpha_extent)
    else:
        arr = oracle.prepare_plain(sc)
        mode = "plain"
        fr = oracle.render(arr, cam, "plain")
    ref = brute_force_image(arr, cam, path, mode, key64, alpha_extent)
    return float(np.max(np.abs(fr.image - ref)))


def check_exact_tile_test(n=2000, seed=5):
    """Share of random (Gaussian, tile) pairs, away from the decision boundary, on which the
    oracle's exact ellipse-tile test disagrees with the least q over a dense grid of the
    tile's box (0 when the closed-form edge minimum is right)."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, 15.0, 121)
    wrong = total = 0
    for _ in range(n):
        L = rng.normal(size=(2, 2)) * rng.choice([1.0, 3.0, 10.0])
        S = L @ L.T + 0.3 * np.eye(2)
        c00, c01, c11 = S[0, 0], S[0, 1], S[1, 1]
        det = c00 * c11 - c01 * c01
        tau = 2.0 * (math.log(255.0) + math.log(rng.uniform(1.0 / 255.0, 1.0)))
        u, v = rng.uniform(-40.0, 56.0, 2)
        dx = xs[None, :] - u
        dy = xs[:, None] - v
        qmin = float(((c11 * dx * dx - 2.0 * c01 * dx * dy + c00 * dy * dy) / det).min())
        if abs(qmin - tau) <= 0.02 * tau + 0.05:
            continue
        total += 1
        keep = bool(oracle.ellipse_meets_tile(u, v, c00, c01, c11, det, tau, 0, 0))
        wrong += keep != (qmin <= tau)
    return wrong / max(total, 1)
