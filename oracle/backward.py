"""Reverse-mode derivative of the plain forward render, in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper renders only; it names training pipelines as where the renderer
would be used next (Sec. V).  This module differentiates the plain image
definition that ``render`` computes (Sec. II-A, III-D; Eqs. alpha_computation,
power, opacity_clamped) with respect to the activated scene parameters:
means, scales, quaternions as given (before normalisation), opacity and SH
coefficients.  Every discrete decision of the forward pass is held fixed:
culling, tile membership, the depth order, the skip test (alpha < 1/255), the
stop test (T (1 - alpha) < 1e-4), the alpha clamp at 0.99 (a clamped alpha has
zero derivative), the clamp of the EWA Jacobian's x/z and y/z at 1.3 tan(fov/2)
and the clamp of each colour channel at 0.  The derivative is the one of the
function those decisions select; finite differences see the same function as
long as no decision flips.

The steps, in reverse order of the forward pass:

* blending (per pixel, over the tile's sorted list):
  C = sum_j c_j alpha_j T_j + T_final bg,  T_j = prod_{i<j} (1 - alpha_i)
  (blended pairs only), so
  dC/dc_j = alpha_j T_j and
  dC/dalpha_j = c_j T_j - (S_j + T_final bg) / (1 - alpha_j),
  S_j = sum_{i>j} c_i alpha_i T_i;
  alpha = o exp(p): dalpha/do = exp(p), dalpha/dp = alpha;
  p = -1/2 (A dx^2 + C dy^2) - B dx dy with (dx, dy) = (x - u, y - v);
* conic (A, B, C) = (c11, -c01, c00) / det, det = c00 c11 - c01^2, with
  (c00, c01, c11) the entries of Sigma';
* Sigma' = T Sigma T^T + 0.3 I with T = J R_w; J from t = R_w mu + t_w (clamped as in
  the forward pass); u = fx t_x / t_z + cx, v = fy t_y / t_z + cy;
* Sigma = M M^T, M = R(q/|q|) diag(s);
* colour_c = max(0, 0.5 + sum_k Y_k(dir) sh_kc), dir = (mu - o_cam)/|mu - o_cam|.

The oracle's forward pass keeps every per-pair quantity, so transmittance is
taken from the forward pass here; the GPU recomputes it instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .blend import ALPHA_MAX, ALPHA_MIN, T_MIN
from .project import J_CLAMP, camera_center, quat_to_rotation, sh_basis
from .render import _tile_pixels, render

# image-space quantities of a Gaussian, in the order the adjoint reports them
SCREEN = ("u", "v", "A", "B", "C", "opacity", "r", "g", "b")


@dataclass
class TileAdjoint:
    grad: np.ndarray       # [n_entries, 9] dL/d(u, v, A, B, C, o, r, g, b), summed over pixels
    abs_sum: np.ndarray    # [n_entries, 9] the same sums of absolute values (conditioning)
    flagged: np.ndarray    # [npix] bool: a decision lies within the margin of its threshold
    entry_flagged: np.ndarray  # [n_entries] bool: blended, or near a decision, at a flagged pixel
    near: list             # (pixel, entry, kind) of every decision within its margin
    terms: np.ndarray      # [n_entries, 9, npix] the per-pixel terms


# Relative margins within which a decision counts as uncertain for a float32
# implementation: alpha carries about 2e-6 relative error (exponent error of a
# few 1e-7 times |p| <= 6), so the skip and clamp tests get 1e-5; T carries the
# error of every (1 - alpha) factor, amplified up to 100x when alpha is near
# 0.99, so the stop test gets 1e-3.
DECISION_MARGINS = (1e-5, 1e-3, 1e-5)      # skip, stop, clamp


def blend_tile_adjoint(gauss_ids, X, Y, u, v, conic, opa, color, bg, dC, margins=DECISION_MARGINS,
                       force=None, flip=None) -> TileAdjoint:
    """dL/d(image-space quantities) of the Gaussians ``gauss_ids`` (sorted) of one tile.

    ``dC`` is dL/d(pixel colour), [3, npix], for pixels at X, Y.  A pixel is
    flagged when one of its skip, stop or clamp decisions lies within the
    relative ``margins`` of its threshold, or when ``force`` [npix] says so.
    ``flip`` = (entry, kind) takes that entry's "skip", "stop" or "clamp"
    decision the other way at every pixel (used one pixel at a time).
    ``margins`` may carry a fourth value kappa: the skip and clamp margins of
    each pair then grow by kappa M, M the magnitude sum of the terms of its
    exponent in coordinates relative to the centre of the pixel's 16x16 tile
    (the folded form of Sec. IV-B, whose float32 evaluation errs by a multiple
    of M; the same M as the forward bookkeeping's tile-centre frame).
    """
    m_skip, m_stop, m_clamp = margins[:3]
    kappa = margins[3] if len(margins) > 3 else 0.0
    near_list = []
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    ids = np.asarray(gauss_ids, np.int64)
    k, n = ids.size, X.size
    # forward pass, keeping every pair's values
    alpha = np.zeros((k, n))
    ep = np.zeros((k, n))
    T_before = np.zeros((k, n))
    blended = np.zeros((k, n), bool)
    clamped = np.zeros((k, n), bool)
    dxs = np.zeros((k, n))
    dys = np.zeros((k, n))
    near = np.zeros((k, n), bool)
    flagged = np.zeros(n, bool)
    T = np.ones(n)
    done = np.zeros(n, bool)
    tcx = np.floor(X / 16.0) * 16.0 + 7.5
    tcy = np.floor(Y / 16.0) * 16.0 + 7.5
    for j, g in enumerate(ids):
        dx = X - u[g]
        dy = Y - v[g]
        A, B, Cc = conic[g]
        p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        ms, mc = m_skip, m_clamp
        if kappa > 0.0:
            ax = np.abs(X - tcx) + np.abs(u[g] - tcx)
            ay = np.abs(Y - tcy) + np.abs(v[g] - tcy)
            lno = np.log(opa[g]) if opa[g] > 0.0 else 0.0
            M = 0.5 * (abs(A) * ax * ax + 2.0 * abs(B) * ax * ay + abs(Cc) * ay * ay) + abs(lno)
            ms, mc = m_skip + kappa * M, m_clamp + kappa * M
        e = np.exp(p)
        raw = opa[g] * e
        a = np.minimum(ALPHA_MAX, raw)
        active = ~done
        pass_test = raw >= ALPHA_MIN
        clamp_test = raw > ALPHA_MAX
        if flip is not None and flip[0] == j and flip[1] == "clamp":
            clamp_test = ~clamp_test
            a = np.where(clamp_test, ALPHA_MAX, raw)
        if flip is not None and flip[0] == j and flip[1] == "skip":
            pass_test = ~pass_test
        passes = active & pass_test
        Tn = T * (1.0 - a)
        stop_test = Tn < T_MIN
        if flip is not None and flip[0] == j and flip[1] == "stop":
            stop_test = ~stop_test
        stop = passes & stop_test
        blend = passes & ~stop
        n_skip = active & (np.abs(raw - ALPHA_MIN) <= ms * ALPHA_MIN)
        n_stop = passes & (np.abs(Tn - T_MIN) <= m_stop * T_MIN)
        n_clamp = passes & (np.abs(raw - ALPHA_MAX) <= mc * ALPHA_MAX)
        for kind, mask in (("skip", n_skip), ("stop", n_stop), ("clamp", n_clamp)):
            for px in np.nonzero(mask)[0]:
                near_list.append((int(px), j, kind))
        nr = n_skip | n_stop | n_clamp
        near[j] = nr
        flagged |= nr
        alpha[j] = np.where(blend, a, 0.0)
        ep[j] = e
        T_before[j] = T
        blended[j] = blend
        clamped[j] = blend & clamp_test
        dxs[j] = dx
        dys[j] = dy
        T = np.where(blend, Tn, T)
        done |= stop
    T_final = T
    if force is not None:
        flagged |= force
    col = color[ids]                                   # [k, 3]
    contrib = alpha[:, None, :] * T_before[:, None, :] * col[:, :, None]      # [k, 3, n]
    # S_j = sum of contributions behind j
    S = np.cumsum(contrib[::-1], axis=0)[::-1] - contrib
    bgT = np.asarray(bg, np.float64)[:, None] * T_final[None, :]             # [3, n]
    one_m = np.where(blended, 1.0 - alpha, 1.0)
    dC_dalpha = col[:, :, None] * T_before[:, None, :] - (S + bgT[None]) / one_m[:, None, :]
    dL_dalpha = np.einsum("kcn,cn->kn", dC_dalpha, dC) * blended
    dL_dcol = (alpha * T_before)[:, None, :] * dC[None]                       # [k, 3, n]
    live = blended & ~clamped
    dL_draw = np.where(live, dL_dalpha, 0.0)           # d alpha / d (o e^p) = 1 when not clamped
    dL_do = dL_draw * ep
    dL_dp = dL_draw * opa[ids][:, None] * ep
    A = conic[ids, 0][:, None]
    B = conic[ids, 1][:, None]
    Cc = conic[ids, 2][:, None]
    terms = np.stack([
        dL_dp * (A * dxs + B * dys),                    # dp/du = A dx + B dy
        dL_dp * (Cc * dys + B * dxs),                   # dp/dv = C dy + B dx
        dL_dp * (-0.5 * dxs * dxs),
        dL_dp * (-dxs * dys),
        dL_dp * (-0.5 * dys * dys),
        dL_do,
        dL_dcol[:, 0], dL_dcol[:, 1], dL_dcol[:, 2],
    ], axis=1)                                          # [k, 9, n]
    # a decision that flips at a pixel changes T after it and S before it: every
    # pair blended there is affected
    entry_flagged = ((blended | near) & flagged[None, :]).any(axis=1)
    return TileAdjoint(grad=terms.sum(axis=2), abs_sum=np.abs(terms).sum(axis=2), flagged=flagged,
                       entry_flagged=entry_flagged, near=near_list, terms=terms)


def sh_basis_jacobian(dirs: np.ndarray) -> np.ndarray:
    """dY_k/d(x, y, z) of the degree-3 basis as polynomials in (x, y, z), [n, 16, 3]."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    pi = math.pi
    n = dirs.shape[0]
    J = np.zeros((n, 16, 3))
    c1 = math.sqrt(3.0 / (4.0 * pi))
    J[:, 1, 1] = -c1
    J[:, 2, 2] = c1
    J[:, 3, 0] = -c1
    c2a = 0.5 * math.sqrt(15.0 / pi)
    c2b = 0.25 * math.sqrt(5.0 / pi)
    c2c = 0.25 * math.sqrt(15.0 / pi)
    J[:, 4, 0], J[:, 4, 1] = c2a * y, c2a * x                     # c2a x y
    J[:, 5, 1], J[:, 5, 2] = -c2a * z, -c2a * y                   # -c2a y z
    J[:, 6, 0], J[:, 6, 1], J[:, 6, 2] = -2 * c2b * x, -2 * c2b * y, 4 * c2b * z
    J[:, 7, 0], J[:, 7, 2] = -c2a * z, -c2a * x                   # -c2a x z
    J[:, 8, 0], J[:, 8, 1] = 2 * c2c * x, -2 * c2c * y            # c2c (x^2 - y^2)
    c3a = 0.25 * math.sqrt(35.0 / (2.0 * pi))
    c3b = 0.5 * math.sqrt(105.0 / pi)
    c3c = 0.25 * math.sqrt(21.0 / (2.0 * pi))
    c3d = 0.25 * math.sqrt(7.0 / pi)
    c3e = 0.25 * math.sqrt(105.0 / pi)
    # -c3a y (3x^2 - y^2)
    J[:, 9, 0], J[:, 9, 1] = -c3a * 6 * x * y, -c3a * (3 * x * x - 3 * y * y)
    # c3b x y z
    J[:, 10, 0], J[:, 10, 1], J[:, 10, 2] = c3b * y * z, c3b * x * z, c3b * x * y
    # -c3c y (4z^2 - x^2 - y^2)
    J[:, 11, 0] = -c3c * y * (-2 * x)
    J[:, 11, 1] = -c3c * (4 * z * z - x * x - 3 * y * y)
    J[:, 11, 2] = -c3c * y * 8 * z
    # c3d z (2z^2 - 3x^2 - 3y^2)
    J[:, 12, 0] = c3d * z * (-6 * x)
    J[:, 12, 1] = c3d * z * (-6 * y)
    J[:, 12, 2] = c3d * (6 * z * z - 3 * x * x - 3 * y * y)
    # -c3c x (4z^2 - x^2 - y^2)
    J[:, 13, 0] = -c3c * (4 * z * z - 3 * x * x - y * y)
    J[:, 13, 1] = -c3c * x * (-2 * y)
    J[:, 13, 2] = -c3c * x * 8 * z
    # c3e z (x^2 - y^2)
    J[:, 14, 0], J[:, 14, 1], J[:, 14, 2] = c3e * z * 2 * x, -c3e * z * 2 * y, c3e * (x * x - y * y)
    # -c3a x (x^2 - 3y^2)
    J[:, 15, 0], J[:, 15, 1] = -c3a * (3 * x * x - 3 * y * y), -c3a * x * (-6 * y)
    return J


def rotation_jacobian(qn: np.ndarray) -> np.ndarray:
    """dR_ab/dq_c of the rotation of a unit quaternion (w, x, y, z) as written in
    ``quat_to_rotation``, [n, 3, 3, 4]."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    n = qn.shape[0]
    D = np.zeros((n, 3, 3, 4))
    W, X_, Y_, Z = 0, 1, 2, 3
    D[:, 0, 0, Y_], D[:, 0, 0, Z] = -4 * y, -4 * z
    D[:, 0, 1, W], D[:, 0, 1, X_], D[:, 0, 1, Y_], D[:, 0, 1, Z] = -2 * z, 2 * y, 2 * x, -2 * w
    D[:, 0, 2, W], D[:, 0, 2, X_], D[:, 0, 2, Y_], D[:, 0, 2, Z] = 2 * y, 2 * z, 2 * w, 2 * x
    D[:, 1, 0, W], D[:, 1, 0, X_], D[:, 1, 0, Y_], D[:, 1, 0, Z] = 2 * z, 2 * y, 2 * x, 2 * w
    D[:, 1, 1, X_], D[:, 1, 1, Z] = -4 * x, -4 * z
    D[:, 1, 2, W], D[:, 1, 2, X_], D[:, 1, 2, Y_], D[:, 1, 2, Z] = -2 * x, -2 * w, 2 * z, 2 * y
    D[:, 2, 0, W], D[:, 2, 0, X_], D[:, 2, 0, Y_], D[:, 2, 0, Z] = -2 * y, 2 * z, -2 * w, 2 * x
    D[:, 2, 1, W], D[:, 2, 1, X_], D[:, 2, 1, Y_], D[:, 2, 1, Z] = 2 * x, 2 * w, 2 * z, 2 * y
    D[:, 2, 2, X_], D[:, 2, 2, Y_] = -4 * x, -4 * y
    return D


@dataclass
class ProjectAdjoint:
    means: np.ndarray     # [n,3]
    scales: np.ndarray    # [n,3]
    quats: np.ndarray     # [n,4]
    opacity: np.ndarray   # [n]
    sh: np.ndarray        # [n,16,3]
    flagged: np.ndarray   # [n] bool: a clamp decision of the front end lies within the margin


def project_adjoint(arrays: dict, cam, visible: np.ndarray, screen_grad: np.ndarray,
                    margin=1e-4) -> ProjectAdjoint:
    """Chain dL/d(u, v, A, B, C, o, r, g, b) [n, 9] back to the activated parameters.

    Only ``visible`` Gaussians carry gradients.  A Gaussian is flagged when
    t_x/t_z or t_y/t_z lies within relative ``margin`` of the Jacobian clamp or
    a colour channel's 0.5 + sum_k Y_k sh_k lies within ``margin`` of 0.
    """
    means = np.asarray(arrays["means"], np.float64)
    quats = np.asarray(arrays["quats"], np.float64)
    scales = np.asarray(arrays["scales"], np.float64)
    sh = np.asarray(arrays["sh"], np.float64)
    n = means.shape[0]
    out = ProjectAdjoint(np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros(n),
                         np.zeros((n, 16, 3)), np.zeros(n, bool))
    idx = np.nonzero(visible)[0]
    if idx.size == 0:
        return out
    mu, q, s, k = means[idx], quats[idx], scales[idx], sh[idx]
    G = screen_grad[idx]
    g_u, g_v, g_A, g_B, g_C, g_o = (G[:, i] for i in range(6))
    g_rgb = G[:, 6:9]
    Rw = np.asarray(cam.R, np.float64)
    tw = np.asarray(cam.t, np.float64)
    fx, fy = cam.fx, cam.fy

    # forward quantities (the forward pass's expression order)
    mx, my, mz = mu[:, 0], mu[:, 1], mu[:, 2]
    tx = Rw[0, 0] * mx + Rw[0, 1] * my + Rw[0, 2] * mz + tw[0]
    ty = Rw[1, 0] * mx + Rw[1, 1] * my + Rw[1, 2] * mz + tw[1]
    d = Rw[2, 0] * mx + Rw[2, 1] * my + Rw[2, 2] * mz + tw[2]
    nq = np.linalg.norm(q, axis=1)
    qn = q / nq[:, None]
    R = quat_to_rotation(qn)
    M = R * s[:, None, :]
    Sig = np.einsum("nak,nbk->nab", M, M)
    limx = J_CLAMP * cam.tan_half_fovx
    limy = J_CLAMP * cam.tan_half_fovy
    rx, ry = tx / d, ty / d
    inx = (rx > -limx) & (rx < limx)
    iny = (ry > -limy) & (ry < limy)
    xc = np.clip(rx, -limx, limx) * d
    yc = np.clip(ry, -limy, limy) * d
    j00, j11 = fx / d, fy / d
    j02 = -fx * xc / (d * d)
    j12 = -fy * yc / (d * d)
    Tm = np.zeros((idx.size, 2, 3))
    Tm[:, 0, :] = j00[:, None] * Rw[0][None, :] + j02[:, None] * Rw[2][None, :]
    Tm[:, 1, :] = j11[:, None] * Rw[1][None, :] + j12[:, None] * Rw[2][None, :]
    cov = np.einsum("nia,nab,njb->nij", Tm, Sig, Tm)
    s00, s01, s11 = cov[:, 0, 0], cov[:, 0, 1], cov[:, 1, 1]
    c00, c11 = s00 + 0.3, s11 + 0.3
    det = c00 * c11 - s01 * s01

    # conic -> Sigma' entries (c00, c01, c11)
    id2 = 1.0 / (det * det)
    g00 = g_A * (-c11 * c11 * id2) + g_B * (s01 * c11 * id2) + g_C * (1.0 / det - c00 * c11 * id2)
    g11 = g_A * (1.0 / det - c11 * c00 * id2) + g_B * (s01 * c00 * id2) + g_C * (-c00 * c00 * id2)
    g01 = (g_A * (2.0 * s01 * c11 * id2) + g_B * (-1.0 / det - 2.0 * s01 * s01 * id2)
           + g_C * (2.0 * c00 * s01 * id2))
    # Sigma' = T Sigma T^T
    T0, T1 = Tm[:, 0, :], Tm[:, 1, :]
    GS = (g00[:, None, None] * T0[:, :, None] * T0[:, None, :]
          + g01[:, None, None] * T0[:, :, None] * T1[:, None, :]
          + g11[:, None, None] * T1[:, :, None] * T1[:, None, :])
    ST0 = np.einsum("nab,nb->na", Sig, T0)
    ST1 = np.einsum("nab,nb->na", Sig, T1)
    gT0 = 2.0 * g00[:, None] * ST0 + g01[:, None] * ST1
    gT1 = 2.0 * g11[:, None] * ST1 + g01[:, None] * ST0
    # T = J R_w
    g_j00 = gT0 @ Rw[0]
    g_j02 = gT0 @ Rw[2]
    g_j11 = gT1 @ Rw[1]
    g_j12 = gT1 @ Rw[2]
    # J and (u, v) -> camera-space t
    g_tx = g_u * fx / d + np.where(inx, g_j02 * (-fx / (d * d)), 0.0)
    g_ty = g_v * fy / d + np.where(iny, g_j12 * (-fy / (d * d)), 0.0)
    g_d = (g_u * (-fx * tx / (d * d)) + g_v * (-fy * ty / (d * d))
           + g_j00 * (-fx / (d * d)) + g_j11 * (-fy / (d * d))
           + g_j02 * np.where(inx, 2.0 * fx * tx / d ** 3, fx * np.sign(rx) * limx / (d * d))
           + g_j12 * np.where(iny, 2.0 * fy * ty / d ** 3, fy * np.sign(ry) * limy / (d * d)))
    g_t = np.stack([g_tx, g_ty, g_d], axis=1)
    g_mu = g_t @ Rw
    # Sigma = M M^T, M = R diag(s)
    gM = np.einsum("nab,nbk->nak", GS + np.transpose(GS, (0, 2, 1)), M)
    g_s = np.einsum("nak,nak->nk", gM, R)
    gR = gM * s[:, None, :]
    g_qn = np.einsum("nab,nabc->nc", gR, rotation_jacobian(qn))
    g_q = (g_qn - qn * np.sum(qn * g_qn, axis=1, keepdims=True)) / nq[:, None]
    # colour
    vdir = mu - camera_center(cam)[None, :]
    vlen = np.linalg.norm(vdir, axis=1)
    dirs = vdir / vlen[:, None]
    Yb = sh_basis(dirs)
    acc = np.einsum("nk,nkc->nc", Yb, k) + 0.5
    m = acc > 0.0
    g_acc = g_rgb * m
    g_sh = Yb[:, :, None] * g_acc[:, None, :]
    g_Y = np.einsum("nkc,nc->nk", k, g_acc)
    g_dir = np.einsum("nk,nkj->nj", g_Y, sh_basis_jacobian(dirs))
    g_mu += (g_dir - dirs * np.sum(dirs * g_dir, axis=1, keepdims=True)) / vlen[:, None]

    out.means[idx] = g_mu
    out.scales[idx] = g_s
    out.quats[idx] = g_q
    out.opacity[idx] = g_o
    out.sh[idx] = g_sh
    near_x = np.abs(np.abs(rx) - limx) <= margin * limx
    near_y = np.abs(np.abs(ry) - limy) <= margin * limy
    near_c = np.any(np.abs(acc) <= margin, axis=1)
    out.flagged[idx] = near_x | near_y | near_c
    return out


@dataclass
class RenderAdjoint:
    image: np.ndarray          # forward image [3, H, W] (NaN outside the tiles)
    screen: np.ndarray         # [n, 9] dL/d(u, v, A, B, C, o, r, g, b)
    screen_abs: np.ndarray     # [n, 9] sums of absolute per-pixel terms
    slack: np.ndarray          # [n, 9] how far decisions near their thresholds can move screen
    params: ProjectAdjoint
    touched: np.ndarray        # [n] bool: blended at some pixel of the tiles
    flagged: np.ndarray        # [n] bool: slack above 1e-3 of screen_abs, or flagged in the front end
    pixel_flagged: np.ndarray  # [H, W] bool
    n_proc: np.ndarray         # [H, W] the oracle's pairs visited per pixel
    n_blend: np.ndarray        # [H, W] the oracle's pairs blended per pixel
    unexplained: int           # pixels whose given decisions differ with no decision near its threshold


def render_adjoint(arrays: dict, cam, dL_dimg: np.ndarray, tiles=None, margins=DECISION_MARGINS,
                   decisions=None) -> RenderAdjoint:
    """Gradients of L with dL/d(image) = ``dL_dimg`` [3, H, W] for the plain path.

    With ``tiles`` given, only those tiles' pixels are differentiated (the
    caller's dL/d(image) must vanish elsewhere).  ``decisions`` = (n_proc,
    n_blend) [H, W] of another implementation's forward pass flags the pixels
    where its pairs visited or blended differ from the oracle's.

    Slack: at each pixel with a decision within its margin, the pixel is
    differentiated again with that decision taken the other way, one decision
    at a time, and the absolute changes of every Gaussian's terms are summed.
    """
    fr = render(arrays, cam, "plain", tiles=tiles)
    force = None
    if decisions is not None:
        force = (np.asarray(decisions[0]) != fr.n_proc) | (np.asarray(decisions[1]) != fr.n_blend)
    plan = fr.plan
    n = arrays["means"].shape[0]
    screen = np.zeros((n, 9))
    screen_abs = np.zeros((n, 9))
    slack = np.zeros((n, 9))
    touched = np.zeros(n, bool)
    loose = np.zeros(n, bool)
    pix_flag = np.zeros((cam.height, cam.width), bool)
    unexplained = 0
    proj = fr.proj
    bg = np.asarray(cam.bg, np.float64)
    opa = arrays["opacity"]
    for t in fr.tiles:
        a, b = fr.ranges[t]
        if b <= a:
            continue
        X, Y = _tile_pixels(int(t), plan)
        Xf, Yf = X.astype(np.float64), Y.astype(np.float64)
        ids = fr.sorted_gauss[a:b]
        dC = dL_dimg[:, Y, X].astype(np.float64)
        fpx = None if force is None else force[Y, X]
        ta = blend_tile_adjoint(ids, Xf, Yf, proj.u, proj.v, proj.conic, opa, proj.color, bg, dC, margins, fpx)
        np.add.at(screen, ids, ta.grad)
        np.add.at(screen_abs, ids, ta.abs_sum)
        hit = ta.abs_sum.sum(axis=1) > 0
        touched[ids[hit]] = True
        pix_flag[Y, X] = ta.flagged
        by_pixel = {}
        for px, j, kind in ta.near:
            by_pixel.setdefault(px, []).append((j, kind))
        if fpx is not None:
            for px in np.nonzero(fpx)[0]:
                if int(px) not in by_pixel:
                    unexplained += 1
                    loose[ids[np.abs(ta.terms[:, :, px]).sum(axis=1) > 0]] = True
        for px, flips in by_pixel.items():
            base = ta.terms[:, :, px]
            dev = np.zeros_like(base)
            for j, kind in flips:
                alt = blend_tile_adjoint(ids, Xf[px:px + 1], Yf[px:px + 1], proj.u, proj.v, proj.conic, opa,
                                         proj.color, bg, dC[:, px:px + 1], margins, None, flip=(j, kind))
                dev += np.abs(alt.terms[:, :, 0] - base)
            np.add.at(slack, ids, dev)
    pa = project_adjoint(arrays, cam, proj.visible, screen)
    flagged = loose | (pa.flagged & touched) | np.any(slack > 1e-3 * screen_abs, axis=1)
    return RenderAdjoint(image=fr.image, screen=screen, screen_abs=screen_abs, slack=slack, params=pa,
                         touched=touched, flagged=flagged, pixel_flagged=pix_flag, n_proc=fr.n_proc,
                         n_blend=fr.n_blend, unexplained=unexplained)


def linear_loss(image: np.ndarray, w: np.ndarray) -> float:
    """sum(w * image): a smooth loss for finite-difference checks."""
    return float(np.sum(w * image))
