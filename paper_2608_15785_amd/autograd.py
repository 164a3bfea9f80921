"""torch.autograd bridge to the plain path's forward and backward passes.

``GaussianRasterizer`` renders a scene whose activated parameters (means,
scales, quaternions, opacity, SH) are torch tensors; the image is
differentiable with respect to all five.  Activations (exp of log-scales,
sigmoid of opacity logits) stay in torch, so their derivatives are torch's.
Every forward call writes the parameters into a device scene (plain format)
and renders into a workspace kept for the backward call; a backward call
whose workspace was used by a later render renders its frame again first.
"""
from __future__ import annotations

import itertools
from types import SimpleNamespace

import numpy as np
import torch

from . import _binding as B
from .renderer import Renderer

_frames = itertools.count(1)


class GaussianRasterizer:
    def __init__(self, renderer: Renderer | None = None, device: int = 0):
        self.R = renderer if renderer is not None else Renderer(device)
        self.scene = None
        self.n = 0
        self._last = {}          # (W, H) -> frame id of the last render into that workspace

    def _scene_for(self, means, scales, quats, opacity, sh):
        n = int(means.shape[0])
        if self.scene is None or self.n != n:
            # the first parameters allocate the device scene; every call rewrites it on the device
            host = SimpleNamespace(means=means.detach().float().cpu().numpy(),
                                   scales=scales.detach().float().cpu().numpy(),
                                   quats=quats.detach().float().cpu().numpy(),
                                   opacity=np.clip(opacity.detach().float().cpu().numpy(), 1e-6, 1.0),
                                   sh=sh.detach().float().cpu().numpy())
            self.scene = self.R.upload(host, ("plain",))
            self.n = n
        return self.scene

    def _render(self, params, cam):
        scene = self._scene_for(*params)
        B.scene_update_plain(self.R.ctx, scene, *(p.detach().float().contiguous() for p in params))
        img, st = self.R.render(scene, cam, "plain")
        fid = next(_frames)
        self._last[(int(cam.width), int(cam.height))] = fid
        return img, fid

    def workspace(self, cam):
        return self.R.workspace(self.n, int(cam.width), int(cam.height), "plain")

    def __call__(self, means, scales, quats, opacity, sh, cam):
        return _RenderFunction.apply(means, scales, quats, opacity, sh, self, cam)


class _RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, rast, cam):
        params = (means, scales, quats, opacity, sh)
        img, fid = rast._render(params, cam)
        ctx.save_for_backward(*params)
        ctx.rast, ctx.cam, ctx.fid = rast, cam, fid
        return img

    @staticmethod
    def backward(ctx, dimg):
        rast, cam = ctx.rast, ctx.cam
        params = ctx.saved_tensors
        if rast._last.get((int(cam.width), int(cam.height))) != ctx.fid:
            rast._render(params, cam)          # the workspace holds another frame: render this one again
        g = B.render_backward(rast.R.ctx, rast.scene, cam, rast.workspace(cam), dimg.float().contiguous())
        return g["means"], g["scales"], g["quats"], g["opacity"], g["sh"], None, None
