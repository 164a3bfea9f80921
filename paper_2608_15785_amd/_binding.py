"""ctypes binding of librgs.so (include/rgs.h): argument marshalling only.

Every step of a render runs in the library's HIP kernels.  torch is used for
device memory (output images, workspaces, parity buffers) and for the current
HIP stream; nothing here computes any part of the render.  If the library is
missing the import fails: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librgs.so")

RGS_OK = 0
RGS_E_INVALID = -1
RGS_E_OOM = -2
RGS_E_HIP = -3
RGS_E_CAPACITY = -4
RGS_E_NODEVICE = -5
RGS_E_UNSUPPORTED = -6
RGS_E_DEVICE = -7

FMT_PLAIN = 1
FMT_FAST = 2
PATH_PLAIN = 0
PATH_FAST = 1
# Ablations of the fast path (rgs.h, RGS_ABLATE_*): a path string
# "fast/no-<name>[/no-<name>...]" removes the named steps.
ABLATIONS = {"fastexp": 1 << 8, "dualpixel": 1 << 9, "fusion": 1 << 10, "extent": 1 << 11,
             "key32": 1 << 12, "int8sh": 1 << 13, "fp16geom": 1 << 14}
# Extensions of the fast path (rgs.h): "fast/<name>" adds them.
EXTENSIONS = {"exact-tiles": 1 << 15, "hw-exp2": 1 << 16, "quad-pixel": 1 << 17}


class _Paths(dict):
    """"plain", "fast", "fast/no-<ablation>/.../<extension>", or "plain/hw-exp2" (the
    plain path's training variant: the dual-pixel rasterizer with folded coefficients,
    culled lists and the hardware exp2 over the plain records, in both passes) -> the C
    path argument."""

    def __missing__(self, key):
        parts = str(key).split("/")
        if parts == ["plain", "hw-exp2"]:
            return PATH_PLAIN | EXTENSIONS["hw-exp2"]
        if parts[0] != "fast" or len(parts) < 2:
            raise KeyError(key)
        code = PATH_FAST
        for p in parts[1:]:
            if p.startswith("no-") and p[3:] in ABLATIONS:
                code |= ABLATIONS[p[3:]]
            elif p in EXTENSIONS:
                code |= EXTENSIONS[p]
            else:
                raise KeyError(key)
        return code


PATHS = _Paths({"plain": PATH_PLAIN, "fast": PATH_FAST})
DEBUG_SORT_FALLBACK = 1
N_STAGES = 5
STAGE_NAMES = ("frontend", "duplicate", "sort", "ranges", "raster")
MAX_ENTRIES = (1 << 30) - 1


class RGSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Plan(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("tiles_x", C.c_int32),
                ("tiles_y", C.c_int32), ("n_tiles", C.c_int32), ("b_t", C.c_int32),
                ("b_d", C.c_int32), ("plain_key_bits", C.c_int32), ("plain_passes", C.c_int32),
                ("fast_passes", C.c_int32)]


class SceneDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32),
                ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class FastHost(C.Structure):
    _fields_ = [("quats_f16", C.c_void_p), ("scales_f16", C.c_void_p), ("lnopa_f16", C.c_void_p),
                ("sh_q", C.c_void_p), ("sh_scale_f16", C.c_void_p)]


class CameraC(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("tan_half_fovx", C.c_double),
                ("tan_half_fovy", C.c_double), ("z_near", C.c_double), ("z_far", C.c_double),
                ("bg", C.c_float * 3), ("reserved", C.c_float)]


class FrameStats(C.Structure):
    _fields_ = [("n_gaussians", C.c_int64), ("n_visible", C.c_int64), ("n_entries", C.c_int64),
                ("capacity", C.c_int64), ("path", C.c_int32), ("passes", C.c_int32),
                ("overflow", C.c_int32), ("device_error", C.c_int32), ("list_steps", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class DebugOut(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("u", C.c_void_p), ("v", C.c_void_p), ("cov2d", C.c_void_p),
                ("rect", C.c_void_p), ("visible", C.c_void_p), ("color", C.c_void_p),
                ("keys_unsorted", C.c_void_p), ("vals_unsorted", C.c_void_p),
                ("keys_sorted", C.c_void_p), ("vals_sorted", C.c_void_p),
                ("entry_capacity", C.c_int64), ("ranges", C.c_void_p), ("T_final", C.c_void_p),
                ("n_proc", C.c_void_p), ("n_blend", C.c_void_p), ("tile_order", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("d_means", C.c_void_p), ("d_scales", C.c_void_p), ("d_quats", C.c_void_p),
                ("d_opacity", C.c_void_p), ("d_sh", C.c_void_p), ("d_screen", C.c_void_p),
                ("scratch", C.c_void_p), ("scratch_bytes", C.c_uint64)]


class DeviceParams(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("n_streams", C.c_int32), ("mem_budget", C.c_uint64),
                ("use_graphs", C.c_int32), ("reserved", C.c_int32), ("entries_per_gaussian", C.c_double)]


class Request(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("camera", CameraC), ("width", C.c_int32), ("height", C.c_int32),
                ("path", C.c_int32), ("reserved", C.c_int32), ("arrival", C.c_double),
                ("out_chw", C.c_void_p)]


class Response(C.Structure):
    _fields_ = [("status", C.c_int32), ("slot", C.c_int32), ("graph", C.c_int32), ("retried", C.c_int32),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("latency", C.c_double),
                ("n_entries", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("wall", C.c_double), ("ws_bytes_held", C.c_uint64), ("ws_bytes_peak", C.c_uint64),
                ("n_workspaces", C.c_int32), ("n_captured", C.c_int32), ("n_evicted", C.c_int32),
                ("max_in_flight", C.c_int32), ("mean_in_flight", C.c_double), ("reserved", C.c_double)]


# (name, restype, argtypes) of every entry point of rgs.h
SIGNATURES = [
    ("rgs_abi_version", C.c_int32, []),
    ("rgs_last_error", C.c_char_p, []),
    ("rgs_status_string", C.c_char_p, [C.c_int32]),
    ("rgs_frame_plan", C.c_int32, [C.c_int32, C.c_int32, C.POINTER(Plan)]),
    ("rgs_ctx_create", C.c_int32, [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("rgs_ctx_destroy", None, [C.c_void_p]),
    ("rgs_ctx_set_stream", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("rgs_ctx_set_timing", C.c_int32, [C.c_void_p, C.c_int32]),
    ("rgs_ctx_collect_timing", C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("rgs_scene_upload", C.c_int32, [C.c_void_p, C.POINTER(SceneDesc), C.c_uint32, C.POINTER(C.c_void_p)]),
    ("rgs_scene_release", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("rgs_scene_info", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_uint32),
                                   C.POINTER(C.c_uint64)]),
    ("rgs_quantize_host", C.c_int32, [C.POINTER(SceneDesc), C.POINTER(FastHost)]),
    ("rgs_workspace_size", C.c_int32, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                       C.POINTER(C.c_uint64)]),
    ("rgs_workspace_capacity", C.c_int32, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                           C.POINTER(C.c_int64)]),
    ("rgs_render_workspace_bound", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                               C.POINTER(C.c_uint64)]),
    ("rgs_scene_device_bytes", C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64)]),
    ("rgs_render", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(CameraC), C.c_int32, C.c_int32,
                               C.c_int32, C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(FrameStats)]),
    ("rgs_workspace_check", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(FrameStats), C.c_int64]),
    ("rgs_render_debug", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(CameraC), C.c_int32, C.c_int32,
                                     C.c_int32, C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(DebugOut),
                                     C.POINTER(FrameStats)]),
    ("rgs_probe_valu", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    ("rgs_ctx_set_debug", C.c_int32, [C.c_void_p, C.c_uint32]),
    ("rgs_render_static", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(CameraC), C.c_int32, C.c_int32,
                                      C.c_int32, C.c_void_p, C.POINTER(FrameStats)]),
    ("rgs_server_create", C.c_int32, [C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]),
    ("rgs_server_destroy", None, [C.c_void_p]),
    ("rgs_serve", C.c_int32, [C.c_void_p, C.POINTER(Request), C.c_int64, C.POINTER(Response),
                              C.POINTER(ServerStats)]),
    ("rgs_scene_update_plain", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(DeviceParams)]),
    ("rgs_backward_scratch_size", C.c_int32, [C.c_int64, C.c_int32, C.c_int32, C.c_uint64,
                                              C.POINTER(C.c_uint64)]),
    ("rgs_render_backward", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(CameraC), C.c_int32, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(Grads)]),
]


def _load():
    # torch bundles its own HIP and HSA runtimes.  Loaded first, they are the
    # process's only ones: librgs.so's libamdhip64.so.7 then resolves to torch's
    # copy.  Loaded after the library, they would come in as a second pair of
    # runtimes beside /opt/rocm's, and the second cannot open the device.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the renderer has no fallback path)")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int, what: str = ""):
    if status != RGS_OK:
        msg = lib.rgs_last_error().decode() or lib.rgs_status_string(status).decode()
        raise RGSError(status, f"{what}: {msg}" if what else msg)


def _ptr(a) -> int | None:
    """Address of a numpy array or torch tensor (None for None)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


# ---------------------------------------------------------------------------
# host-only calls

def frame_plan(width: int, height: int) -> dict:
    p = Plan()
    _check(lib.rgs_frame_plan(width, height, C.byref(p)), "rgs_frame_plan")
    return {k: getattr(p, k) for k, _ in Plan._fields_}


def _scene_arrays(scene):
    arrs = dict(means=np.ascontiguousarray(scene.means, np.float32),
                scales=np.ascontiguousarray(scene.scales, np.float32),
                quats=np.ascontiguousarray(scene.quats, np.float32),
                opacity=np.ascontiguousarray(scene.opacity, np.float32),
                sh=np.ascontiguousarray(scene.sh, np.float32))
    n = arrs["means"].shape[0]
    desc = SceneDesc(n, 3, 0, *(arrs[k].ctypes.data for k in ("means", "scales", "quats", "opacity", "sh")))
    return desc, arrs


def quantize_host(scene) -> dict:
    """The library's compact storage of a scene (FP16 bit patterns as uint16)."""
    desc, keep = _scene_arrays(scene)
    n = desc.n
    out = dict(quats=np.zeros((n, 4), np.uint16), scales=np.zeros((n, 3), np.uint16),
               log_opacity=np.zeros(n, np.uint16), sh_q=np.zeros((n, 16, 3), np.int8),
               sh_scale=np.zeros((n, 4, 3), np.uint16))
    fh = FastHost(*(out[k].ctypes.data for k in ("quats", "scales", "log_opacity", "sh_q", "sh_scale")))
    _check(lib.rgs_quantize_host(C.byref(desc), C.byref(fh)), "rgs_quantize_host")
    return out


def workspace_size(n: int, width: int, height: int, path: str, max_entries: int) -> int:
    b = C.c_uint64()
    _check(lib.rgs_workspace_size(n, width, height, PATHS[path], max_entries, C.byref(b)),
           "rgs_workspace_size")
    return int(b.value)


def workspace_capacity(n: int, width: int, height: int, path: str, ws_bytes: int) -> int:
    c = C.c_int64()
    _check(lib.rgs_workspace_capacity(n, width, height, PATHS[path], ws_bytes, C.byref(c)),
           "rgs_workspace_capacity")
    return int(c.value)


def camera_struct(cam) -> CameraC:
    c = CameraC()
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
        c.bg[k] = float(np.asarray(cam.bg, np.float32)[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.tan_half_fovx, c.tan_half_fovy = float(cam.tan_half_fovx), float(cam.tan_half_fovy)
    c.z_near, c.z_far = float(cam.z_near), float(cam.z_far)
    c.reserved = 0.0
    return c


# ---------------------------------------------------------------------------
# device calls

def _torch():
    import torch
    return torch


def probe_valu(ctx: "Context", blocks: int, iters: int, out) -> None:
    """Enqueues the VALU calibration probe (rgs_probe_valu): blocks x 256
    threads, 8 * iters FMA instructions per wave; out is a float32 device
    tensor of at least blocks * 256 elements."""
    if out.numel() < blocks * 256 or out.dtype != _torch().float32 or not out.is_cuda:
        raise ValueError("out must be a float32 device tensor of blocks * 256 elements")
    _check(lib.rgs_probe_valu(ctx.handle, int(blocks), int(iters), _ptr(out)), "rgs_probe_valu")


class Context:
    """A device and a stream (torch's current stream unless one is given)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.device = device
        h = C.c_void_p()
        if stream is None and _torch().cuda.is_available():
            stream = _torch().cuda.current_stream(device).cuda_stream
        _check(lib.rgs_ctx_create(device, stream, C.byref(h)), "rgs_ctx_create")
        self.handle = h.value

    def set_stream(self, stream: int):
        _check(lib.rgs_ctx_set_stream(self.handle, stream), "rgs_ctx_set_stream")

    def set_debug(self, flags: int):
        """RGS_DEBUG_* flags for this context's renders (DEBUG_SORT_FALLBACK)."""
        _check(lib.rgs_ctx_set_debug(self.handle, int(flags)), "rgs_ctx_set_debug")

    def set_timing(self, on: bool):
        _check(lib.rgs_ctx_set_timing(self.handle, 1 if on else 0), "rgs_ctx_set_timing")

    def collect_timing(self):
        ms = (C.c_double * N_STAGES)()
        n = C.c_int64()
        _check(lib.rgs_ctx_collect_timing(self.handle, ms, C.byref(n)), "rgs_ctx_collect_timing")
        return dict(zip(STAGE_NAMES, list(ms))), int(n.value)

    def close(self):
        if self.handle:
            lib.rgs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceScene:
    """A scene uploaded to the context's device in the plain and/or fast format."""

    def __init__(self, ctx: Context, scene, formats=("plain", "fast")):
        fm = (FMT_PLAIN if "plain" in formats else 0) | (FMT_FAST if "fast" in formats else 0)
        desc, keep = _scene_arrays(scene)
        h = C.c_void_p()
        _check(lib.rgs_scene_upload(ctx.handle, C.byref(desc), fm, C.byref(h)), "rgs_scene_upload")
        self.ctx = ctx
        self.handle = h.value
        self.n = int(desc.n)

    def info(self) -> dict:
        n, f, b = C.c_int64(), C.c_uint32(), C.c_uint64()
        _check(lib.rgs_scene_info(self.handle, C.byref(n), C.byref(f), C.byref(b)), "rgs_scene_info")
        return dict(n=int(n.value), formats=int(f.value), device_bytes=int(b.value))

    def device_bytes(self) -> int:
        b = C.c_uint64()
        _check(lib.rgs_scene_device_bytes(self.handle, C.byref(b)), "rgs_scene_device_bytes")
        return int(b.value)

    def workspace_bound(self, width: int, height: int, path: str, hint_ndup: int = 0) -> int:
        """Workspace bytes a render of this scene needs for hint_ndup entries (0: the default guess)."""
        b = C.c_uint64()
        _check(lib.rgs_render_workspace_bound(self.handle, width, height, PATHS[path], hint_ndup, C.byref(b)),
               "rgs_render_workspace_bound")
        return int(b.value)

    def release(self):
        if self.handle:
            lib.rgs_scene_release(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def new_workspace(n: int, width: int, height: int, path: str, max_entries: int, device: int = 0):
    torch = _torch()
    nbytes = workspace_size(n, width, height, path, max_entries)
    return torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{device}")


STATIC_WORKSPACE_BYTES = 128 << 20


def render_static(ctx: Context, scene: DeviceScene, cam, path: str, out=None, stats: bool = False):
    """rgs_render_static: one render into the library's static workspace (nothing is
    allocated by the call; ``out``, if given, is the caller's image)."""
    torch = _torch()
    W, H = int(cam.width), int(cam.height)
    if out is None:
        out = torch.empty((3, H, W), dtype=torch.float32, device=f"cuda:{ctx.device}")
    cc = camera_struct(cam)
    st = FrameStats() if stats else None
    _check(lib.rgs_render_static(ctx.handle, scene.handle, C.byref(cc), W, H, PATHS[path], out.data_ptr(),
                                 C.byref(st) if st is not None else None), "rgs_render_static")
    return out, (st.as_dict() if st is not None else None)


def render(ctx: Context, scene: DeviceScene, cam, path: str, workspace, out=None, stats: bool = False):
    """Enqueue one render; returns (image [3,H,W] float32 tensor, stats dict or None)."""
    torch = _torch()
    W, H = int(cam.width), int(cam.height)
    if out is None:
        out = torch.empty((3, H, W), dtype=torch.float32, device=workspace.device)
    cc = camera_struct(cam)
    st = FrameStats() if stats else None
    _check(lib.rgs_render(ctx.handle, scene.handle, C.byref(cc), W, H, PATHS[path], workspace.data_ptr(),
                          workspace.numel(), out.data_ptr(), C.byref(st) if st is not None else None),
           "rgs_render")
    return out, (st.as_dict() if st is not None else None)


class Server:
    """Continuous-batching request server over resident scenes (``rgs_serve``)."""

    def __init__(self, device: int = 0, n_streams: int = 4, mem_budget: int = 8 << 30,
                 use_graphs: bool = True, entries_per_gaussian: float = 0.0):
        cfg = ServerConfig(device=device, n_streams=n_streams, mem_budget=int(mem_budget),
                           use_graphs=1 if use_graphs else 0, reserved=0,
                           entries_per_gaussian=float(entries_per_gaussian))
        h = C.c_void_p()
        _check(lib.rgs_server_create(C.byref(cfg), C.byref(h)), "rgs_server_create")
        self.handle = h.value

    def serve(self, requests):
        """Run a schedule.  ``requests``: sequence of (DeviceScene, camera, path, arrival_s, out) with
        ``out`` a device tensor [3, H, W]; returns (list of response dicts, stats dict)."""
        n = len(requests)
        reqs = (Request * max(n, 1))()
        for i, (scene, cam, path, arrival, out) in enumerate(requests):
            r = reqs[i]
            r.scene = scene.handle
            r.camera = camera_struct(cam)
            r.width, r.height = int(cam.width), int(cam.height)
            r.path = PATHS[path]
            r.reserved = 0
            r.arrival = float(arrival)
            r.out_chw = out.data_ptr()
        resp = (Response * max(n, 1))()
        st = ServerStats()
        _check(lib.rgs_serve(self.handle, reqs, n, resp, C.byref(st)), "rgs_serve")
        rows = [{k: getattr(resp[i], k) for k, _ in Response._fields_} for i in range(n)]
        return rows, {k: getattr(st, k) for k, _ in ServerStats._fields_ if k != "reserved"}

    def close(self):
        if self.handle:
            lib.rgs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_stats(ctx: Context, workspace, n: int = 0) -> dict:
    """Statistics of the last frame rendered into ``workspace``, whatever its status."""
    st = FrameStats()
    status = lib.rgs_workspace_check(ctx.handle, workspace.data_ptr(), C.byref(st), n)
    if status not in (RGS_OK, RGS_E_CAPACITY, RGS_E_DEVICE):
        _check(status, "rgs_workspace_check")
    return st.as_dict()


def workspace_check(ctx: Context, workspace, n: int = 0) -> dict:
    st = FrameStats()
    _check(lib.rgs_workspace_check(ctx.handle, workspace.data_ptr(), C.byref(st), n), "rgs_workspace_check")
    return st.as_dict()


def render_debug(ctx: Context, scene: DeviceScene, cam, path: str, workspace, entry_capacity: int):
    """Render and return the frame's intermediates as numpy arrays."""
    torch = _torch()
    dev = workspace.device
    W, H = int(cam.width), int(cam.height)
    n = scene.n
    t = dict(
        depth=torch.zeros(n, dtype=torch.float64, device=dev),
        u=torch.zeros(n, dtype=torch.float64, device=dev),
        v=torch.zeros(n, dtype=torch.float64, device=dev),
        cov2d=torch.zeros((n, 3), dtype=torch.float64, device=dev),
        rect=torch.zeros((n, 4), dtype=torch.int32, device=dev),
        visible=torch.zeros(n, dtype=torch.uint8, device=dev),
        color=torch.zeros((n, 3), dtype=torch.float32, device=dev),
        keys_unsorted=torch.zeros(entry_capacity, dtype=torch.int64, device=dev),
        vals_unsorted=torch.zeros(entry_capacity, dtype=torch.int32, device=dev),
        keys_sorted=torch.zeros(entry_capacity, dtype=torch.int64, device=dev),
        vals_sorted=torch.zeros(entry_capacity, dtype=torch.int32, device=dev),
        ranges=torch.zeros((frame_plan(W, H)["n_tiles"], 2), dtype=torch.int32, device=dev),
        T_final=torch.zeros((H, W), dtype=torch.float32, device=dev),
        n_proc=torch.zeros((H, W), dtype=torch.int32, device=dev),
        n_blend=torch.zeros((H, W), dtype=torch.int32, device=dev),
        tile_order=torch.zeros(frame_plan(W, H)["n_tiles"], dtype=torch.int32, device=dev),
    )
    image = torch.zeros((3, H, W), dtype=torch.float32, device=dev)
    dbg = DebugOut(*(_ptr(t[k]) for k in ("depth", "u", "v", "cov2d", "rect", "visible", "color",
                                          "keys_unsorted", "vals_unsorted", "keys_sorted", "vals_sorted")),
                   entry_capacity, *(_ptr(t[k]) for k in ("ranges", "T_final", "n_proc", "n_blend", "tile_order")))
    cc = camera_struct(cam)
    st = FrameStats()
    _check(lib.rgs_render_debug(ctx.handle, scene.handle, C.byref(cc), W, H, PATHS[path],
                                workspace.data_ptr(), workspace.numel(), image.data_ptr(),
                                C.byref(dbg), C.byref(st)), "rgs_render_debug")
    torch.cuda.synchronize(dev)
    out = {k: v.cpu().numpy() for k, v in t.items()}
    m = int(st.n_entries)
    for k in ("keys_unsorted", "keys_sorted"):
        out[k] = out[k][:m].view(np.uint64)
    for k in ("vals_unsorted", "vals_sorted"):
        out[k] = out[k][:m].view(np.uint32)
    out["ranges"] = out["ranges"].view(np.uint32)
    word = out["n_proc"].view(np.uint32)
    out["n_proc"] = word & np.uint32(0x7FFFFFFF)          # pairs visited
    out["stopped"] = (word >> np.uint32(31)).astype(bool)  # blending stopped at the last of them
    out["n_blend"] = out["n_blend"].view(np.uint32)
    out["tile_order"] = out["tile_order"].view(np.uint32)
    out["visible"] = out["visible"].astype(bool)
    out["image"] = image.cpu().numpy()
    out["stats"] = st.as_dict()
    return out


def scene_update_plain(ctx: Context, scene: DeviceScene, means, scales, quats, opacity, sh):
    """Overwrite the plain attributes of ``scene`` from contiguous float32 device tensors."""
    for t in (means, scales, quats, opacity, sh):
        if not (t.is_contiguous() and t.dtype == _torch().float32 and t.is_cuda):
            raise ValueError("parameters must be contiguous float32 device tensors")
    p = DeviceParams(n=int(means.shape[0]), means=means.data_ptr(), scales=scales.data_ptr(),
                     quats=quats.data_ptr(), opacity=opacity.data_ptr(), sh=sh.data_ptr())
    _check(lib.rgs_scene_update_plain(ctx.handle, scene.handle, C.byref(p)), "rgs_scene_update_plain")


def backward_scratch_size(n: int, width: int, height: int, ws_bytes: int) -> int:
    b = C.c_uint64()
    _check(lib.rgs_backward_scratch_size(n, width, height, ws_bytes, C.byref(b)), "rgs_backward_scratch_size")
    return int(b.value)


def render_backward(ctx: Context, scene: DeviceScene, cam, workspace, dL_dimg, scratch=None,
                    screen: bool = False) -> dict:
    """Gradients w.r.t. the activated plain parameters after a plain render into ``workspace``.

    Returns float32 device tensors means [n,3], scales [n,3], quats [n,4], opacity [n], sh [n,16,3]
    (and screen [n,9] = dL/d(u, v, A, B, C, o, r, g, b) when ``screen``)."""
    torch = _torch()
    n = scene.n
    W, H = int(cam.width), int(cam.height)
    dev = workspace.device
    need = backward_scratch_size(n, W, H, workspace.numel())
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    g = dict(means=torch.empty((n, 3), dtype=torch.float32, device=dev),
             scales=torch.empty((n, 3), dtype=torch.float32, device=dev),
             quats=torch.empty((n, 4), dtype=torch.float32, device=dev),
             opacity=torch.empty((n,), dtype=torch.float32, device=dev),
             sh=torch.empty((n, 16, 3), dtype=torch.float32, device=dev))
    if screen:
        g["screen"] = torch.empty((n, 9), dtype=torch.float32, device=dev)
    dimg = dL_dimg.contiguous()
    if dimg.shape != (3, H, W) or dimg.dtype != torch.float32:
        raise ValueError("dL_dimg must be float32 [3, H, W]")
    gr = Grads(d_means=g["means"].data_ptr(), d_scales=g["scales"].data_ptr(), d_quats=g["quats"].data_ptr(),
               d_opacity=g["opacity"].data_ptr(), d_sh=g["sh"].data_ptr(),
               d_screen=g["screen"].data_ptr() if screen else None, scratch=scratch.data_ptr(),
               scratch_bytes=scratch.numel())
    cc = camera_struct(cam)
    _check(lib.rgs_render_backward(ctx.handle, scene.handle, C.byref(cc), W, H, dimg.data_ptr(),
                                   workspace.data_ptr(), workspace.numel(), C.byref(gr)), "rgs_render_backward")
    return g
