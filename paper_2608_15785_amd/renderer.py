"""Workspace management around the C ABI: one context, scenes, and a workspace
per (scene size, resolution, path) that grows when a frame reports overflow."""
from __future__ import annotations

from . import _binding as B


class Renderer:
    def __init__(self, device: int = 0, stream: int | None = None):
        self.device = device
        self.ctx = B.Context(device, stream)
        self._ws = {}

    def upload(self, scene, formats=("plain", "fast")) -> B.DeviceScene:
        return B.DeviceScene(self.ctx, scene, formats)

    def workspace(self, n: int, width: int, height: int, path: str, min_entries: int | None = None):
        key = (n, width, height, path)
        ws = self._ws.get(key)
        want = min_entries if min_entries is not None else max(4 * n, 1 << 16)
        want = min(want, B.MAX_ENTRIES)
        if ws is None or B.workspace_capacity(n, width, height, path, ws.numel()) < want:
            ws = B.new_workspace(n, width, height, path, want, self.device)
            self._ws[key] = ws
        return ws

    def render(self, dscene: B.DeviceScene, cam, path: str, out=None, check: bool = True):
        """Render one frame.  check=True synchronises, grows the workspace and
        re-renders if the frame overflowed, and returns the frame statistics."""
        W, H = int(cam.width), int(cam.height)
        ws = self.workspace(dscene.n, W, H, path)
        if not check:
            img, _ = B.render(self.ctx, dscene, cam, path, ws, out)
            return img, None
        for _ in range(4):
            try:
                return B.render(self.ctx, dscene, cam, path, ws, out, stats=True)
            except B.RGSError as e:
                if e.status != B.RGS_E_CAPACITY:
                    raise
                need = self._needed(ws, dscene.n)
                ws = self.workspace(dscene.n, W, H, path, int(need * 1.25) + 4096)
        raise RuntimeError("workspace growth did not converge")

    def _needed(self, ws, n: int) -> int:
        """Entries the last frame in ``ws`` asked for (its header keeps the count)."""
        return int(B.workspace_stats(self.ctx, ws, n)["n_entries"])

    def check(self, dscene: B.DeviceScene, cam, path: str) -> dict:
        ws = self.workspace(dscene.n, int(cam.width), int(cam.height), path)
        return B.workspace_check(self.ctx, ws, dscene.n)

    def render_debug(self, dscene: B.DeviceScene, cam, path: str):
        W, H = int(cam.width), int(cam.height)
        img, st = self.render(dscene, cam, path)
        need = int(st["n_entries"])
        ws = self.workspace(dscene.n, W, H, path, max(need, 1))
        return B.render_debug(self.ctx, dscene, cam, path, ws, max(need, 1))
