"""torch.autograd bridge to the plain path's forward and backward passes.

``GaussianRasterizer`` renders a scene whose activated parameters (means,
scales, quaternions, opacity, SH) are torch tensors; the image is
differentiable with respect to all five.  Activations (exp of log-scales,
sigmoid of opacity logits) stay in torch, so their derivatives are torch's.

Every forward call writes the parameters into the rasterizer's device scene
(plain format) and renders into a workspace the rasterizer owns for that image
size, which no other renderer writes.  A backward call differentiates the
frame its forward produced: when the workspace has seen a later frame, or the
device scene has been rewritten since (a forward at another size, or with
other parameters), it renders its own frame again first.  The library checks
the same thing on its side (the workspace records which scene state, camera
and size its last frame came from) and refuses a mismatch.
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
    """hw_exp2=True renders and differentiates with the plain path's training
    variant ("plain/hw-exp2": the dual-pixel rasterizer with folded coefficients,
    culled lists and the hardware exp2, in both passes)."""

    def __init__(self, renderer: Renderer | None = None, device: int = 0, hw_exp2: bool = False):
        self.R = renderer if renderer is not None else Renderer(device)
        self.path = "plain/hw-exp2" if hw_exp2 else "plain"
        self.scene = None
        self.n = 0
        self._gen = 0            # parameter writes into the device scene so far
        self._ws = {}            # (W, H) -> this rasterizer's own workspace
        self._last = {}          # (W, H) -> (frame id, scene generation) of the last render there

    def _scene_for(self, means, scales, quats, opacity, sh):
        n = int(means.shape[0])
        if self.scene is None or self.n != n:
            # the first parameters allocate the device scene; every call rewrites it on the device
            host = SimpleNamespace(means=means.detach().float().cpu().numpy(),
                                   scales=scales.detach().float().cpu().numpy(),
                                   quats=quats.detach().float().cpu().numpy(),
                                   opacity=np.clip(opacity.detach().float().cpu().numpy(), 1e-6, 1.0),
                                   sh=sh.detach().float().cpu().numpy())
            if self.scene is not None:
                self.scene.release()
            self.scene = self.R.upload(host, ("plain",))
            self.n = n
            self._ws.clear()
            self._last.clear()
        return self.scene

    def workspace(self, cam, min_entries: int | None = None):
        key = (int(cam.width), int(cam.height))
        ws = self._ws.get(key)
        want = min(min_entries if min_entries is not None else max(4 * self.n, 1 << 16), B.MAX_ENTRIES)
        if ws is None or B.workspace_capacity(self.n, key[0], key[1], "plain", ws.numel()) < want:
            ws = B.new_workspace(self.n, key[0], key[1], "plain", want, self.R.device)
            self._ws[key] = ws
        return ws

    def _render(self, params, cam):
        scene = self._scene_for(*params)
        B.scene_update_plain(self.R.ctx, scene, *(p.detach().float().contiguous() for p in params))
        self._gen += 1
        ws = self.workspace(cam)
        for _ in range(4):
            try:
                img, _ = B.render(self.R.ctx, scene, cam, self.path, ws, stats=True)
                break
            except B.RGSError as e:
                if e.status != B.RGS_E_CAPACITY:
                    raise
                need = int(B.workspace_stats(self.R.ctx, ws, self.n)["n_entries"])
                ws = self.workspace(cam, int(need * 1.25) + 4096)
        else:
            raise RuntimeError("workspace growth did not converge")
        fid = next(_frames)
        self._last[(int(cam.width), int(cam.height))] = (fid, self._gen)
        return img, fid

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
        if rast._last.get((int(cam.width), int(cam.height))) != (ctx.fid, rast._gen):
            # the workspace holds a later frame, or the scene was rewritten since: render this frame again
            rast._render(params, cam)
        g = B.render_backward(rast.R.ctx, rast.scene, cam, rast.workspace(cam), dimg.float().contiguous())
        return g["means"], g["scales"], g["quats"], g["opacity"], g["sh"], None, None
