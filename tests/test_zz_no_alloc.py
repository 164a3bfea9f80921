"""The allocation-free render (rgs_render_static) through the C ABI (needs an MI355X).

Two calls in a row, the second with a smaller input (fewer Gaussians, a smaller
image), and then the first again: each image must equal, bit for bit, the one
rgs_render gives for the same frame in a caller-owned workspace (the same
kernels run on the same inputs; only where the frame's transients live
differs).  A frame whose fixed part cannot fit the static workspace is refused
before any work."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_15785_amd as rgs
    return rgs.Renderer(0)


@pytest.mark.parametrize("path", ["fast", "plain"])
def test_static_render_matches_render(R, path):
    import torch
    from paper_2608_15785_amd import _binding as B
    big = (wl.config_scene("1080p", n=300_000), wl.config_camera("1080p"))
    small = (wl.config_scene("small"), wl.config_camera("small", width=200, height=136))
    dev = {id(big[0]): R.upload(big[0], (path,)), id(small[0]): R.upload(small[0], (path,))}
    for k, (sc, cam) in enumerate((big, small, big)):
        ds = dev[id(sc)]
        _log(f"[static] call {k}: {path} n={sc.n} {cam.width}x{cam.height}")
        out = torch.full((3, cam.height, cam.width), float("nan"), dtype=torch.float32, device="cuda:0")
        img_s, st_s = B.render_static(R.ctx, ds, cam, path, out=out, stats=True)
        torch.cuda.synchronize()
        got = img_s.cpu().numpy().copy()
        ref, st_r = R.render(ds, cam, path)
        torch.cuda.synchronize()
        ref = ref.cpu().numpy()
        assert st_s["overflow"] == 0 and st_s["device_error"] == 0, st_s
        assert st_s["n_entries"] == st_r["n_entries"] and st_s["n_visible"] == st_r["n_visible"]
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), \
            f"static and workspace renders differ at {int(np.count_nonzero(got != ref))} values"
    for ds in dev.values():
        ds.release()


def test_static_render_refuses_a_frame_that_cannot_fit(R):
    import torch
    import paper_2608_15785_amd as rgs
    from paper_2608_15785_amd import _binding as B
    sc = wl.config_scene("small", n=100)
    ds = R.upload(sc, ("fast",))
    cam = wl.config_camera("small", width=8192, height=8192)       # 768 MiB of per-pixel buffers
    out = torch.empty((3, 8192, 8192), dtype=torch.float32, device="cuda:0")   # a real image, though unused
    with pytest.raises(rgs.RGSError) as e:
        cc = B.camera_struct(cam)
        B._check(B.lib.rgs_render_static(R.ctx.handle, ds.handle, B.C.byref(cc), 8192, 8192, B.PATHS["fast"],
                                         out.data_ptr(), None), "rgs_render_static")
    assert e.value.status == B.RGS_E_INVALID and "static workspace" in str(e.value)
    ds.release()
