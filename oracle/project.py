"""Per-Gaussian front end in float64: EWA projection, culling, tile extents, SH colour.

Sec. II-A and III-A describe the preprocess stage (following 3DGS): each 3D
Gaussian (mean mu, rotation r, scale s, opacity o) is projected to a 2D mean
mu' and covariance Sigma', whose inverse (the conic) the rasterizer evaluates
(Eq. alpha_computation).  Sec. IV-A adds frustum culling against the
predefined depth interval [z_near, z_far] before key generation, and opacity
culling of Gaussians whose contribution is negligible before duplication.

The paper is silent on the projection's constants and follows 3DGS; the
readings used here are the 3DGS conventions:

* view transform t = R_w mu + t_w, depth d = t_z (camera looks along +z);
* Sigma = R(q) diag(s)^2 R(q)^T with R(q) the rotation of the normalised
  quaternion q = (w, x, y, z);
* the EWA Jacobian J = [[fx/d, 0, -fx x~/d^2], [0, fy/d, -fy y~/d^2]] with
  x~ = clamp(t_x/d, +-1.3 tan(fovx/2)) d (same for y~ with fovy);
* Sigma' = J R_w Sigma R_w^T J^T + 0.3 I (low-pass dilation);
* conic (A, B, C) = (Sigma'_11, -Sigma'_01, Sigma'_00) / det(Sigma'), so that
  the quadratic form of Eq. power is A dx^2 + 2 B dx dy + C dy^2 (the paper's
  b is 2B);
* u = fx t_x / d + cx, v = fy t_y / d + cy.

Culling and extent (readings):

* a Gaussian is culled if d <= z_near or d > z_far, if det(Sigma') <= 0, or if
  its tile rectangle is empty;
* plain extent: a square of half-size r = ceil(3 sqrt(lambda_max(Sigma')));
* fast extent (opacity culling in the spirit of Speedy-Splat): cull when
  o < 1/255 (ln o < -ln 255); otherwise the half-extents are those of the
  box around the ellipse where o exp(p) >= 1/255, tau = 2 (ln 255 + ln o),
  h_x = min(r, sqrt(tau Sigma'_00)), h_y = min(r, sqrt(tau Sigma'_11)).
  Pixels outside that ellipse have alpha < 1/255 and are skipped by the
  rasterizer anyway, so this shrinks the tile set without changing the image;
* tiles x in [max(0, floor((u-h)/16)), min(T_x-1, floor((u+h)/16))], same in y.

Every key-defining quantity (d, u, v, Sigma', the extents) is computed with
the elementwise float64 operations below, evaluated left to right exactly as
written, with no fused multiply-add; division and square root are the
correctly rounded IEEE operations.  The HIP front end evaluates the same
expressions in the same order, so both sides produce identical bits.  The
paper fixes no evaluation order; ours divides once for 1/d and once for the
quaternion's 1/|q| and multiplies them in (mathematically the definitions
above).

SH colour (Sec. III-A, degree 3): view-dependent RGB from 16 coefficients per
channel, evaluated along the unit direction from the camera centre to the
mean, plus 0.5 and clamped at 0 (3DGS convention).  The real SH basis carries
the Condon-Shortley phase, ordered m = -l..l at index l*l + l + m.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .plan import TILE, FramePlan

LN255 = math.log(255.0)
DILATION = 0.3
J_CLAMP = 1.3


@dataclass
class Projection:
    """Per-Gaussian front-end results (float64 unless stated)."""
    d: np.ndarray        # camera-space depth
    u: np.ndarray        # projected mean, pixels
    v: np.ndarray
    cov: np.ndarray      # [n,3] Sigma'_00, Sigma'_01, Sigma'_11
    det: np.ndarray
    conic: np.ndarray    # [n,3] A, B, C
    radius: np.ndarray   # 3-sigma half-size r (integer valued)
    rect: np.ndarray     # [n,4] int64 x0, x1, y0, y1 tile bounds (inclusive)
    visible: np.ndarray  # bool
    color: np.ndarray    # [n,3] RGB (computed for visible Gaussians, else 0)


def quat_to_rotation(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [n,3,3] of quaternions q = (w, x, y, z), normalised first."""
    qw, qx, qy, qz = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    inn = 1.0 / np.sqrt(qw * qw + qx * qx + qy * qy + qz * qz)
    w = qw * inn
    x = qx * inn
    y = qy * inn
    z = qz * inn
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1.0 - 2.0 * (y * y + z * z)
    R[:, 0, 1] = 2.0 * (x * y - w * z)
    R[:, 0, 2] = 2.0 * (x * z + w * y)
    R[:, 1, 0] = 2.0 * (x * y + w * z)
    R[:, 1, 1] = 1.0 - 2.0 * (x * x + z * z)
    R[:, 1, 2] = 2.0 * (y * z - w * x)
    R[:, 2, 0] = 2.0 * (x * z - w * y)
    R[:, 2, 1] = 2.0 * (y * z + w * x)
    R[:, 2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return R


def covariance3d(quats: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """Sigma = M M^T with M = R(q) diag(s); returns [n,3,3]."""
    R = quat_to_rotation(quats)
    M = R * scales[:, None, :]                 # M_ik = R_ik s_k
    S = np.empty_like(M)
    for i in range(3):
        for j in range(3):
            S[:, i, j] = M[:, i, 0] * M[:, j, 0] + M[:, i, 1] * M[:, j, 1] + M[:, i, 2] * M[:, j, 2]
    return S


def project_ewa(means, quats, scales, cam):
    """Camera-space depth, 2D mean and 2D covariance (EWA splatting).

    Returns (tx, ty, d, u, v, cov00, cov01, cov11) as float64 arrays.
    """
    r = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    mx, my, mz = means[:, 0], means[:, 1], means[:, 2]
    tx = r[0, 0] * mx + r[0, 1] * my + r[0, 2] * mz + t[0]
    ty = r[1, 0] * mx + r[1, 1] * my + r[1, 2] * mz + t[1]
    d = r[2, 0] * mx + r[2, 1] * my + r[2, 2] * mz + t[2]

    S = covariance3d(quats, scales)

    limx = J_CLAMP * cam.tan_half_fovx
    limy = J_CLAMP * cam.tan_half_fovy
    rd = 1.0 / d
    rd2 = rd * rd
    xc = np.minimum(limx, np.maximum(-limx, tx * rd)) * d
    yc = np.minimum(limy, np.maximum(-limy, ty * rd)) * d
    j00 = cam.fx * rd
    j02 = -(cam.fx * xc) * rd2
    j11 = cam.fy * rd
    j12 = -(cam.fy * yc) * rd2

    # T = J R_w (2x3); J has zeros at (0,1) and (1,0)
    T = np.empty((means.shape[0], 2, 3))
    for k in range(3):
        T[:, 0, k] = j00 * r[0, k] + j02 * r[2, k]
        T[:, 1, k] = j11 * r[1, k] + j12 * r[2, k]
    # U = T Sigma, then Sigma' = U T^T + 0.3 I
    U = np.empty_like(T)
    for i in range(2):
        for k in range(3):
            U[:, i, k] = T[:, i, 0] * S[:, 0, k] + T[:, i, 1] * S[:, 1, k] + T[:, i, 2] * S[:, 2, k]
    cov00 = U[:, 0, 0] * T[:, 0, 0] + U[:, 0, 1] * T[:, 0, 1] + U[:, 0, 2] * T[:, 0, 2] + DILATION
    cov01 = U[:, 0, 0] * T[:, 1, 0] + U[:, 0, 1] * T[:, 1, 1] + U[:, 0, 2] * T[:, 1, 2]
    cov11 = U[:, 1, 0] * T[:, 1, 0] + U[:, 1, 1] * T[:, 1, 1] + U[:, 1, 2] * T[:, 1, 2] + DILATION

    u = cam.fx * tx * rd + cam.cx
    v = cam.fy * ty * rd + cam.cy
    return tx, ty, d, u, v, cov00, cov01, cov11


def tile_rect(u, v, hx, hy, plan: FramePlan) -> np.ndarray:
    """Inclusive tile bounds [x0, x1, y0, y1] of the box u +- hx, v +- hy."""
    x0 = np.maximum(0.0, np.floor((u - hx) / TILE))
    x1 = np.minimum(plan.tiles_x - 1.0, np.floor((u + hx) / TILE))
    y0 = np.maximum(0.0, np.floor((v - hy) / TILE))
    y1 = np.minimum(plan.tiles_y - 1.0, np.floor((v + hy) / TILE))
    return np.stack([x0, x1, y0, y1], axis=1)


def sh_basis(dirs: np.ndarray) -> np.ndarray:
    """Real SH basis Y_lm(dir), degree <= 3, [n,16], for unit directions [n,3]."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    pi = math.pi
    Y = np.empty((dirs.shape[0], 16))
    Y[:, 0] = 0.5 / math.sqrt(pi)
    c1 = math.sqrt(3.0 / (4.0 * pi))
    Y[:, 1] = -c1 * y
    Y[:, 2] = c1 * z
    Y[:, 3] = -c1 * x
    c2a = 0.5 * math.sqrt(15.0 / pi)
    c2b = 0.25 * math.sqrt(5.0 / pi)
    c2c = 0.25 * math.sqrt(15.0 / pi)
    Y[:, 4] = c2a * x * y
    Y[:, 5] = -c2a * y * z
    Y[:, 6] = c2b * (2.0 * z * z - x * x - y * y)
    Y[:, 7] = -c2a * x * z
    Y[:, 8] = c2c * (x * x - y * y)
    c3a = 0.25 * math.sqrt(35.0 / (2.0 * pi))
    c3b = 0.5 * math.sqrt(105.0 / pi)
    c3c = 0.25 * math.sqrt(21.0 / (2.0 * pi))
    c3d = 0.25 * math.sqrt(7.0 / pi)
    c3e = 0.25 * math.sqrt(105.0 / pi)
    Y[:, 9] = -c3a * y * (3.0 * x * x - y * y)
    Y[:, 10] = c3b * x * y * z
    Y[:, 11] = -c3c * y * (4.0 * z * z - x * x - y * y)
    Y[:, 12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y)
    Y[:, 13] = -c3c * x * (4.0 * z * z - x * x - y * y)
    Y[:, 14] = c3e * z * (x * x - y * y)
    Y[:, 15] = -c3a * x * (x * x - 3.0 * y * y)
    return Y


def camera_center(cam) -> np.ndarray:
    """World position of the camera centre, -R^T t."""
    return -np.asarray(cam.R, np.float64).T @ np.asarray(cam.t, np.float64)


def sh_color(means, sh, cam) -> np.ndarray:
    """RGB = max(0, 0.5 + sum_k Y_k(dir) sh_k) with dir from the camera to the mean."""
    dirs = means - camera_center(cam)[None, :]
    dirs = dirs / np.linalg.norm(dirs, axis=1, keepdims=True)
    Y = sh_basis(dirs)
    rgb = np.einsum("nk,nkc->nc", Y, sh) + 0.5
    return np.maximum(rgb, 0.0)


def project(arrays: dict, cam, plan: FramePlan, fast: bool, alpha_extent: bool = True) -> Projection:
    """The whole per-Gaussian front end for the plain (fast=False) or fast path.

    ``arrays`` holds float64 means [n,3], quats [n,4], scales [n,3], sh
    [n,16,3] and either ``opacity`` [n] (plain) or ``log_opacity`` [n] (fast).
    ``alpha_extent=False`` drops the fast path's opacity cull and alpha-ellipse
    extent and keeps the 3-sigma square (the ablation of that step).
    """
    means, quats, scales = arrays["means"], arrays["quats"], arrays["scales"]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        tx, ty, d, u, v, c00, c01, c11 = project_ewa(means, quats, scales, cam)
        det = c00 * c11 - c01 * c01
        conic = np.stack([c11 / det, -c01 / det, c00 / det], axis=1)
        mid = 0.5 * (c00 + c11)
        lam = mid + np.sqrt(np.maximum(0.0, mid * mid - det))
        r = np.ceil(3.0 * np.sqrt(lam))
        visible = (d > cam.z_near) & (d <= cam.z_far) & (det > 0.0)
        if fast and alpha_extent:
            lno = arrays["log_opacity"]
            visible &= lno >= -LN255
            tau = 2.0 * (LN255 + lno)
            hx = np.minimum(r, np.sqrt(tau * c00))
            hy = np.minimum(r, np.sqrt(tau * c11))
        else:
            hx = r
            hy = r
        rect = tile_rect(u, v, hx, hy, plan)
    visible &= (rect[:, 0] <= rect[:, 1]) & (rect[:, 2] <= rect[:, 3])
    rect = np.where(visible[:, None], rect, 0.0).astype(np.int64)
    color = np.zeros((means.shape[0], 3))
    if visible.any():
        color[visible] = sh_color(means[visible], arrays["sh"][visible], cam)
    return Projection(d=d, u=u, v=v, cov=np.stack([c00, c01, c11], axis=1), det=det,
                      conic=conic, radius=r, rect=rect, visible=visible, color=color)
