"""Backward pass of the plain render through the C ABI against the FP64 oracle
adjoint (needs an MI355X).

The oracle's adjoint is pinned to finite differences of its forward render on
the CPU.  Here the GPU's gradients (image-space per Gaussian, then the
activated parameters) are compared with it Gaussian by Gaussian.

Tolerances.  Each image-space derivative of a Gaussian is a sum of per-pixel
terms computed in float32 with transmittance recovered by division; its error
is bounded by 1e-3 of the sum of the terms' magnitudes (the oracle reports that
sum).  Where a skip, stop or clamp decision lies near its threshold, float32
and float64 may take it differently; the oracle differentiates those pixels
again with the decision flipped and adds the change of every Gaussian's terms
as slack.  Every Gaussian the loss reaches is checked to that bound.  The
parameter gradients are the double-precision chain rule applied to those
sums; they are checked, for the Gaussians whose slack is below 1e-3 of their
terms, to 2e-3 of the largest gradient of their kind plus 2e-3 of themselves.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import backward as OB

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


PATHS = ["plain", "plain/hw-exp2"]      # the plain path and its training variant
# The training variant evaluates each exponent in the folded form of Sec. IV-B
# (tile-centre coordinates, float32), whose error scales with the magnitude sum
# M of its terms: its skip and clamp margins grow by 4e-6 M per pair, as the
# fast path's forward bookkeeping does.
MARGINS = {"plain": OB.DECISION_MARGINS, "plain/hw-exp2": OB.DECISION_MARGINS + (4e-6,)}


def gpu_backward(R, scene, cam, dimg, path="plain"):
    import torch
    import paper_2608_15785_amd as rgs
    ds = R.upload(scene, ("plain",))
    dbg = R.render_debug(ds, cam, path)           # the frame, with its per-pixel decisions
    ws = R.workspace(scene.n, cam.width, cam.height, path)
    g = rgs.render_backward(R.ctx, ds, cam, ws, torch.from_numpy(dimg).cuda(), screen=True)
    torch.cuda.synchronize()
    chk = rgs.workspace_check(R.ctx, ws, scene.n)
    assert chk["device_error"] == 0, chk
    out = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    out["image"] = dbg["image"]
    out["decisions"] = (dbg["n_proc"].astype(np.int64), dbg["n_blend"].astype(np.int64))
    ds.release()
    return out


def compare(g, adj, n_expect_min=1):
    touched = adj.touched
    strict = touched & ~adj.flagged
    _log(f"[bwd] flagged pixels {int(adj.pixel_flagged.sum())}, touched {int(touched.sum())}, "
         f"strict {int(strict.sum())}, with slack {int(adj.flagged.sum())}")
    assert adj.unexplained == 0, "GPU decisions differ where no decision is near its threshold"
    assert strict.sum() >= n_expect_min
    assert adj.flagged.sum() <= 0.1 * max(1, touched.sum()), "too many near-threshold decisions"
    # untouched Gaussians: exactly zero
    for k in ("means", "scales", "quats", "opacity", "sh", "screen"):
        assert np.all(g[k][~touched] == 0.0), k
    # image-space sums, every touched Gaussian
    err = np.abs(g["screen"][touched] - adj.screen[touched])
    bound = 1e-3 * adj.screen_abs[touched] + adj.slack[touched] + 1e-7
    worst = float(np.max(err / bound)) if err.size else 0.0
    _log(f"[bwd] screen: worst err/bound {worst:.3g}")
    assert np.all(err <= bound), np.unravel_index(np.argmax(err / bound), err.shape)
    # parameter gradients
    p = adj.params
    ref = dict(means=p.means, scales=p.scales, quats=p.quats, opacity=p.opacity, sh=p.sh)
    for k, o in ref.items():
        gv = g[k][strict]
        ov = o[strict]
        scale = np.max(np.abs(ov)) if ov.size else 0.0
        e = np.abs(gv - ov)
        tol = 2e-3 * scale + 2e-3 * np.abs(ov)
        rel = float(np.linalg.norm(gv - ov) / max(np.linalg.norm(ov), 1e-30))
        _log(f"[bwd] {k}: max err {float(e.max()):.3g} (scale {scale:.3g}), rel L2 {rel:.3g}")
        assert np.all(e <= tol + 1e-12), (k, float(e.max()))
        assert rel < 1e-3, (k, rel)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("W,H", [(128, 96), (120, 88)])
def test_small_scene_all_tiles(R, W, H, path):
    sc = wl.make_scene(3000, 1.0, -3.0, 0.5, 31)
    cam = wl.config_camera("small", width=W, height=H)
    cam.bg = np.array([0.1, 0.2, 0.3], np.float32)
    rng = np.random.Generator(np.random.PCG64(41))
    dimg = rng.normal(0.0, 1.0, (3, H, W)).astype(np.float32)
    _log(f"[bwd] small scene n={sc.n} {W}x{H} {path}")
    g = gpu_backward(R, sc, cam, dimg, path)
    adj = OB.render_adjoint(oracle.prepare_plain(sc), cam, dimg.astype(np.float64), margins=MARGINS[path],
                            decisions=g["decisions"])
    compare(g, adj, n_expect_min=1000)


def test_deterministic(R):
    sc = wl.make_scene(2000, 1.0, -3.0, 0.5, 32)
    cam = wl.config_camera("small", width=96, height=80)
    dimg = np.random.Generator(np.random.PCG64(3)).normal(0, 1, (3, 80, 96)).astype(np.float32)
    a = gpu_backward(R, sc, cam, dimg)
    b = gpu_backward(R, sc, cam, dimg)
    for k in ("means", "scales", "quats", "opacity", "sh", "screen"):
        assert np.array_equal(a[k], b[k]), k
    assert np.abs(a["screen"]).sum() > 0


@pytest.mark.parametrize("path", PATHS)
def test_training_l1_loss_sampled_tiles(R, path):
    """1M Gaussians at 1080p; L1 loss against a render of the same scene with
    means perturbed by N(0, 0.01); dL/d(image) kept on 40 sampled tiles so that
    the oracle differentiates exactly the same loss."""
    import torch
    sc = wl.config_scene("1080p")
    cam = wl.config_camera("1080p")
    H, W = cam.height, cam.width
    target_scene = wl.Scene(means=wl.perturbed_means(sc), scales=sc.scales, quats=sc.quats,
                            opacity=sc.opacity, sh=sc.sh)
    dt = R.upload(target_scene, ("plain",))
    target, _ = R.render(dt, cam, "plain")
    torch.cuda.synchronize()
    target = target.cpu().numpy()
    dt.release()
    ds = R.upload(sc, ("plain",))
    img, _ = R.render(ds, cam, path)
    torch.cuda.synchronize()
    img = img.cpu().numpy()
    ds.release()
    plan = oracle.frame_plan(W, H)
    rng = np.random.Generator(np.random.PCG64(4))
    tiles = np.sort(rng.choice(plan.n_tiles, 40, replace=False))
    mask = np.zeros((H, W), bool)
    for t in tiles:
        tx, ty = t % plan.tiles_x, t // plan.tiles_x
        mask[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = True
    dimg = (np.sign(img - target) / img.size * mask[None]).astype(np.float32)
    _log(f"[bwd] training ({path}): L1 loss {np.abs(img - target).mean():.6g}, {len(tiles)} tiles")
    g = gpu_backward(R, sc, cam, dimg, path)
    assert np.array_equal(g["image"], img)
    adj = OB.render_adjoint(oracle.prepare_plain(sc), cam, dimg.astype(np.float64), tiles=tiles,
                            margins=MARGINS[path], decisions=g["decisions"])
    compare(g, adj, n_expect_min=2000)


def test_autograd_function_chains_activations(R):
    import torch
    from paper_2608_15785_amd.autograd import GaussianRasterizer
    import paper_2608_15785_amd as rgs
    sc = wl.make_scene(1500, 1.0, -3.0, 0.5, 33)
    cam = wl.config_camera("small", width=64, height=64)
    dev = "cuda:0"
    means = torch.tensor(sc.means, device=dev, requires_grad=True)
    log_scales = torch.tensor(np.log(sc.scales.astype(np.float64)).astype(np.float32), device=dev,
                              requires_grad=True)
    quats = torch.tensor(sc.quats, device=dev, requires_grad=True)
    o = np.clip(sc.opacity.astype(np.float64), 1e-6, 1 - 1e-6)
    logits = torch.tensor(np.log(o / (1 - o)).astype(np.float32), device=dev, requires_grad=True)
    sh = torch.tensor(sc.sh, device=dev, requires_grad=True)
    rast = GaussianRasterizer(R)
    target = torch.zeros((3, 64, 64), device=dev)
    scales, opac = torch.exp(log_scales), torch.sigmoid(logits)
    img = rast(means, scales, quats, opac, sh, cam)
    loss = (img - target).abs().mean()
    loss.backward()
    # the same gradients straight from the C ABI, chained by hand
    dimg = torch.sign(img.detach() - target) / img.numel()
    ws = rast.workspace(cam)
    g = rgs.render_backward(R.ctx, rast.scene, cam, ws, dimg)
    torch.cuda.synchronize()
    assert torch.equal(means.grad, g["means"])
    assert torch.equal(quats.grad, g["quats"])
    assert torch.equal(sh.grad, g["sh"])
    assert torch.allclose(log_scales.grad, g["scales"] * scales.detach(), rtol=1e-6, atol=0)
    assert torch.allclose(logits.grad, g["opacity"] * opac.detach() * (1 - opac.detach()), rtol=1e-6, atol=0)
    # a small step against the gradient lowers the loss
    with torch.no_grad():
        for p in (means, log_scales, quats, logits, sh):
            p -= 1e-3 * p.grad / (p.grad.abs().max() + 1e-30)
        img2 = rast(means, torch.exp(log_scales), quats, torch.sigmoid(logits), sh, cam)
        assert (img2 - target).abs().mean() < loss


def test_backward_refuses_a_fast_frame_and_small_scratch(R):
    import torch
    import paper_2608_15785_amd as rgs
    from paper_2608_15785_amd import _binding as B
    sc = wl.make_scene(500, 1.0, -3.0, 0.5, 34)
    cam = wl.config_camera("small", width=48, height=32)
    ds = R.upload(sc)
    dimg = torch.zeros((3, 32, 48), device="cuda:0")
    R.render(ds, cam, "fast")
    ws_fast = R.workspace(sc.n, 48, 32, "fast")
    with pytest.raises(rgs.RGSError) as e:
        rgs.render_backward(R.ctx, ds, cam, ws_fast, dimg)
    assert e.value.status == B.RGS_E_INVALID
    R.render(ds, cam, "plain")
    ws = R.workspace(sc.n, 48, 32, "plain")
    tiny = torch.empty(256, dtype=torch.uint8, device="cuda:0")
    need = rgs.backward_scratch_size(sc.n, 48, 32, ws.numel())
    assert need > 256
    with pytest.raises(rgs.RGSError) as e:
        g = rgs.render_backward(R.ctx, ds, cam, ws, dimg, scratch=None)
        # a scratch buffer that is too small is replaced by the binding; call the ABI directly
        gr = B.Grads(d_means=g["means"].data_ptr(), d_scales=g["scales"].data_ptr(),
                     d_quats=g["quats"].data_ptr(), d_opacity=g["opacity"].data_ptr(), d_sh=g["sh"].data_ptr(),
                     d_screen=None, scratch=tiny.data_ptr(), scratch_bytes=256)
        cc = B.camera_struct(cam)
        B._check(B.lib.rgs_render_backward(R.ctx.handle, ds.handle, B.C.byref(cc), 48, 32, dimg.data_ptr(),
                                           ws.data_ptr(), ws.numel(), B.C.byref(gr)), "rgs_render_backward")
    assert e.value.status == B.RGS_E_INVALID
    torch.cuda.synchronize()
    ds.release()


@pytest.mark.parametrize("path", PATHS)
def test_backward_refuses_an_overflowed_frame(R, path):
    """A frame that overflowed its workspace has no complete lists to differentiate: the
    backward call reports RGS_E_CAPACITY (from the frame's stamp, which the calling context
    rendered), and again when asked through the workspace header (a workspace another
    context rendered)."""
    import torch
    import paper_2608_15785_amd as rgs
    from paper_2608_15785_amd import _binding as B
    sc = wl.make_scene(2000, 1.0, -3.0, 0.5, 43)
    cam = wl.config_camera("small", width=128, height=96)
    ds = R.upload(sc, ("plain",))
    dimg = torch.ones((3, 96, 128), device="cuda:0")
    ws = B.new_workspace(sc.n, 128, 96, "plain", 64, 0)        # far fewer entries than the frame has
    out = torch.empty((3, 96, 128), device="cuda:0")
    B.render(R.ctx, ds, cam, path, ws, out)
    with pytest.raises(rgs.RGSError) as e:
        rgs.render_backward(R.ctx, ds, cam, ws, dimg)
    assert e.value.status == B.RGS_E_CAPACITY
    R2 = rgs.Renderer(0)
    with pytest.raises(rgs.RGSError) as e:
        rgs.render_backward(R2.ctx, ds, cam, ws, dimg)
    assert e.value.status == B.RGS_E_CAPACITY
    torch.cuda.synchronize()
    del R2
    ds.release()


def test_backward_refuses_a_stale_workspace(R):
    """The workspace records which scene state, camera and size its last frame
    came from; the backward call refuses any other frame."""
    import torch
    import paper_2608_15785_amd as rgs
    from paper_2608_15785_amd import _binding as B
    sc = wl.make_scene(500, 1.0, -3.0, 0.5, 35)
    other = wl.make_scene(500, 1.0, -3.0, 0.5, 36)
    cam = wl.config_camera("small", width=48, height=32)
    cam2 = wl.look_at_camera((0.3, 0.1, -3.0), (0, 0, 0), (0, 1, 0), 60.0, 48, 32, cam.z_near, cam.z_far)
    ds, ds2 = R.upload(sc, ("plain",)), R.upload(other, ("plain",))
    dimg = torch.ones((3, 32, 48), device="cuda:0")
    ws = R.workspace(sc.n, 48, 32, "plain")
    R.render(ds, cam, "plain")
    rgs.render_backward(R.ctx, ds, cam, ws, dimg)              # the frame it holds: accepted
    R.render(ds2, cam, "plain")                                # another scene into the same workspace
    assert R.workspace(sc.n, 48, 32, "plain").data_ptr() == ws.data_ptr()
    with pytest.raises(rgs.RGSError) as e:
        rgs.render_backward(R.ctx, ds, cam, ws, dimg)
    assert e.value.status == B.RGS_E_INVALID and "scene" in str(e.value)
    R.render(ds, cam, "plain")
    with pytest.raises(rgs.RGSError) as e:                     # another camera of the same size
        rgs.render_backward(R.ctx, ds, cam2, ws, dimg)
    assert e.value.status == B.RGS_E_INVALID and "camera" in str(e.value)
    params = [torch.tensor(np.ascontiguousarray(a, np.float32), device="cuda:0")
              for a in (sc.means, sc.scales, sc.quats, sc.opacity, sc.sh)]
    rgs.scene_update_plain(R.ctx, ds, *params)                 # same values, but a new scene state
    with pytest.raises(rgs.RGSError) as e:
        rgs.render_backward(R.ctx, ds, cam, ws, dimg)
    assert e.value.status == B.RGS_E_INVALID
    R.render(ds, cam, "plain")
    rgs.render_backward(R.ctx, ds, cam, ws, dimg)
    torch.cuda.synchronize()
    ds.release()
    ds2.release()


@pytest.mark.parametrize("n", [1000, 4099])
def test_scene_update_equals_upload(R, n):
    """rgs_scene_update_plain writes the same planes as an upload of the same parameters:
    a scene uploaded from other values, updated, renders like a fresh upload (a full block
    of 256 Gaussians and a ragged last one).  Bit for bit on the plain path; the training
    variant also reads ln o, which the upload takes from the host's log and the update from
    the device's (both in float64, rounded to float32), so it may differ by an ulp there."""
    import torch
    import paper_2608_15785_amd as rgs
    a = wl.make_scene(n, 1.0, -3.0, 0.5, 41)
    b = wl.make_scene(n, 1.0, -3.0, 0.5, 42)
    cam = wl.config_camera("small", width=128, height=96)
    for path in ("plain", "plain/hw-exp2"):
        ds_b = R.upload(b, ("plain",))
        ref, _ = R.render(ds_b, cam, path)
        ref = ref.clone()
        ds_b.release()
        ds = R.upload(a, ("plain",))
        params = [torch.tensor(np.ascontiguousarray(x, np.float32), device="cuda:0")
                  for x in (b.means, b.scales, b.quats, b.opacity, b.sh)]
        rgs.scene_update_plain(R.ctx, ds, *params)
        img, _ = R.render(ds, cam, path)
        torch.cuda.synchronize()
        if path == "plain":
            assert torch.equal(img, ref)
        else:
            assert float((img - ref).abs().max()) <= 1e-5, path
        ds.release()


def test_backward_finds_another_contexts_frame(R):
    """A context differentiates the frame it last rendered into a workspace from that
    frame's stamp, without reading the device.  If another context has rendered another
    frame into the same workspace since, the backward kernels find the workspace's frame
    parameters different from the caller's: they write zero gradients and flag the
    workspace (device error bit 3), which the next check reports."""
    import torch
    import paper_2608_15785_amd as rgs
    from paper_2608_15785_amd import _binding as B
    sc = wl.make_scene(500, 1.0, -3.0, 0.5, 37)
    cam = wl.config_camera("small", width=48, height=32)
    cam2 = wl.look_at_camera((0.3, 0.1, -3.0), (0, 0, 0), (0, 1, 0), 60.0, 48, 32, cam.z_near, cam.z_far)
    ds = R.upload(sc, ("plain",))
    dimg = torch.ones((3, 32, 48), device="cuda:0")
    ws = R.workspace(sc.n, 48, 32, "plain")
    out = torch.empty((3, 32, 48), device="cuda:0")
    B.render(R.ctx, ds, cam, "plain", ws, out)
    g = rgs.render_backward(R.ctx, ds, cam, ws, dimg, screen=True)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(g["screen"])) > 0
    assert B.workspace_stats(R.ctx, ws, sc.n)["device_error"] == 0
    R2 = rgs.Renderer(0)
    B.render(R2.ctx, ds, cam2, "plain", ws, out)               # another context, another camera
    g = rgs.render_backward(R.ctx, ds, cam, ws, dimg, screen=True)
    torch.cuda.synchronize()
    for k, v in g.items():
        assert int(torch.count_nonzero(v)) == 0, k
    st = B.workspace_stats(R.ctx, ws, sc.n)
    assert st["device_error"] & 8, st
    with pytest.raises(rgs.RGSError) as e:
        rgs.workspace_check(R.ctx, ws, sc.n)
    assert e.value.status == B.RGS_E_DEVICE
    B.render(R.ctx, ds, cam, "plain", ws, out)                 # a new frame clears the flag
    g = rgs.render_backward(R.ctx, ds, cam, ws, dimg, screen=True)
    torch.cuda.synchronize()
    assert B.workspace_stats(R.ctx, ws, sc.n)["device_error"] == 0
    assert int(torch.count_nonzero(g["screen"])) > 0
    del R2
    ds.release()


def test_autograd_gradients_survive_interleaved_renders(R):
    """Between a forward call and its backward: a render of another scene of the
    same size through the shared renderer, or a forward at another image size
    with other parameters, leave the gradients bit for bit as they are without
    them."""
    import torch
    from paper_2608_15785_amd.autograd import GaussianRasterizer
    sc = wl.make_scene(1200, 1.0, -3.0, 0.5, 37)
    other = wl.make_scene(1200, 1.0, -3.0, 0.5, 38)
    cam = wl.config_camera("small", width=64, height=64)
    cam_b = wl.config_camera("small", width=80, height=48)
    dev = "cuda:0"
    leaves = [torch.tensor(np.ascontiguousarray(a, np.float32), device=dev, requires_grad=True)
              for a in (sc.means, sc.scales, sc.quats, sc.opacity, sc.sh)]
    rast = GaussianRasterizer(R)

    def loss_of(img):
        return (img - 0.25).abs().mean()

    def grads():
        g = [p.grad.detach().clone() for p in leaves]
        for p in leaves:
            p.grad = None
        return g

    loss_of(rast(*leaves, cam)).backward()
    ref = grads()
    # another scene of the same size rendered through the renderer in between
    ds_other = R.upload(other, ("plain",))
    img = rast(*leaves, cam)
    R.render(ds_other, cam, "plain")
    loss_of(img).backward()
    for a, b in zip(grads(), ref):
        assert torch.equal(a, b)
    # a forward at another size with other parameters in between
    img = rast(*leaves, cam)
    with torch.no_grad():
        moved = [p.detach() + 0.01 if k == 0 else p.detach() for k, p in enumerate(leaves)]
    rast(*moved, cam_b)
    loss_of(img).backward()
    for a, b in zip(grads(), ref):
        assert torch.equal(a, b)
    ds_other.release()
