"""Compact attribute storage of the fast path (Sec. IV-A, "Compact Attribute Storage").

* SH coefficients are stored as INT8 with a symmetric scale for each SH degree
  d in {0,1,2,3} and colour channel c (Eq. quant): s = max|SH| / 127,
  q = round(SH / s), reconstructed as s * q.
  Reading of the scope of the max (the equation leaves it open): per Gaussian,
  per (degree, channel), over the coefficients of that degree, which gives 12
  scales per Gaussian.  Each scale is stored as FP16 (round-to-nearest-even)
  and q is computed against the stored scale, so reconstruction uses exactly
  the value held in memory.  round() is round-half-to-even; q is clamped to
  [-127, 127]; a zero scale gives q = 0.
* Rotation, scale and opacity are stored in FP16 and the mean stays FP32.
  Opacity is held as its logarithm, ln o, computed in float64 from the FP32
  opacity and rounded to FP16: the rasterizer folds ln o into the exponent
  (Eq. coeff, C_6) and opacity culling compares ln o with -ln 255, so no
  transcendental function is evaluated per frame.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# SH coefficient index ranges per degree: l*l .. (l+1)*(l+1)-1
DEGREE_SLICES = [slice(0, 1), slice(1, 4), slice(4, 9), slice(9, 16)]


@dataclass
class FastScene:
    """The fast-path scene exactly as stored (before dequantisation)."""
    means: np.ndarray        # [n,3] float32
    quats: np.ndarray        # [n,4] float16 (w, x, y, z)
    scales: np.ndarray       # [n,3] float16
    log_opacity: np.ndarray  # [n]   float16
    sh_q: np.ndarray         # [n,16,3] int8
    sh_scale: np.ndarray     # [n,4,3] float16, per (degree, channel)


def quantize_sh(sh: np.ndarray):
    """Eq. quant per Gaussian, degree and channel.  Returns (q int8, scale fp16)."""
    sh = np.asarray(sh, np.float64)
    n = sh.shape[0]
    q = np.zeros((n, 16, 3), np.int8)
    scales = np.zeros((n, 4, 3), np.float16)
    for d, sl in enumerate(DEGREE_SLICES):
        block = sh[:, sl, :]                                  # [n, 2d+1, 3]
        s = (np.max(np.abs(block), axis=1) / 127.0).astype(np.float16)   # [n, 3]
        scales[:, d, :] = s
        s64 = s.astype(np.float64)[:, None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(s64 > 0.0, block / s64, 0.0)
        q[:, sl, :] = np.clip(np.rint(ratio), -127, 127).astype(np.int8)
    return q, scales


def dequantize_sh(q: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """Reconstructed coefficients s * q in float64 ([n,16,3])."""
    out = np.zeros(q.shape, np.float64)
    for d, sl in enumerate(DEGREE_SLICES):
        out[:, sl, :] = q[:, sl, :].astype(np.float64) * scales[:, d, None, :].astype(np.float64)
    return out


def quantize_scene(scene) -> FastScene:
    """Build the fast-path storage of a float32 scene."""
    q, s = quantize_sh(scene.sh)
    return FastScene(
        means=np.asarray(scene.means, np.float32),
        quats=np.asarray(scene.quats, np.float32).astype(np.float16),
        scales=np.asarray(scene.scales, np.float32).astype(np.float16),
        log_opacity=np.log(np.asarray(scene.opacity, np.float64)).astype(np.float16),
        sh_q=q,
        sh_scale=s,
    )


def dequantize_scene(fs: FastScene) -> dict:
    """float64 arrays of the stored fast scene, as the fast path computes with them."""
    return dict(
        means=fs.means.astype(np.float64),
        quats=fs.quats.astype(np.float64),
        scales=fs.scales.astype(np.float64),
        log_opacity=fs.log_opacity.astype(np.float64),
        sh=dequantize_sh(fs.sh_q, fs.sh_scale),
    )
