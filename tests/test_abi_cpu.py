"""The C-ABI library on the CPU: it loads, exports every declared entry point,
and its host-only logic (frame plan, workspace sizing, compact-storage
quantiser, argument checks) matches the oracle.  No GPU work is launched."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2608_15785_amd as rgs
import workloads as wl
from paper_2608_15785_amd import _binding as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rgs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rgs_status|int32_t|const char\*|void)\s+(rgs_\w+)\s*\(",
                                 text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 18
    lib = C.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert {n for n, _, _ in B.SIGNATURES} == set(names)
    assert B.lib.rgs_abi_version() == 2


@pytest.mark.parametrize("W,H", [(1, 1), (16, 16), (17, 1), (256, 256), (1280, 720), (1920, 1080),
                                 (3840, 2160), (64, 64), (250, 170), (16384, 16384)])
def test_frame_plan_matches_oracle(W, H):
    p = rgs.frame_plan(W, H)
    o = oracle.frame_plan(W, H)
    assert (p["tiles_x"], p["tiles_y"], p["n_tiles"], p["b_t"], p["b_d"]) == \
        (o.tiles_x, o.tiles_y, o.n_tiles, o.b_t, o.b_d)
    assert p["plain_key_bits"] == o.plain_key_bits
    assert p["plain_passes"] == -(-o.plain_key_bits // 8) and p["fast_passes"] == 4


@pytest.mark.parametrize("W,H", [(0, 10), (10, 0), (-1, 5), (16385, 16), (16, 16385)])
def test_frame_plan_rejects(W, H):
    with pytest.raises(rgs.RGSError) as e:
        rgs.frame_plan(W, H)
    assert e.value.status == B.RGS_E_INVALID


def test_workspace_sizing():
    for path in ("plain", "fast"):
        sizes = [rgs.workspace_size(10_000, 256, 256, path, m) for m in (1, 1000, 100_000, 1_000_000)]
        assert sizes == sorted(sizes) and sizes[0] < sizes[-1]
        for m in (1, 4095, 4096, 4097, 123_457):
            b = rgs.workspace_size(10_000, 256, 256, path, m)
            assert rgs.workspace_capacity(10_000, 256, 256, path, b) >= m
            assert rgs.workspace_capacity(10_000, 256, 256, path, b - 256) < m or m == 1
        assert rgs.workspace_capacity(10_000, 256, 256, path, 1000) == 0
    # the plain entry (64-bit key + index, double-buffered) costs more than the fast one
    assert rgs.workspace_size(1, 16, 16, "plain", 1 << 20) > rgs.workspace_size(1, 16, 16, "fast", 1 << 20)
    for bad in (0, B.MAX_ENTRIES + 1):
        with pytest.raises(rgs.RGSError):
            rgs.workspace_size(10, 16, 16, "fast", bad)


def test_path_words_are_validated():
    """Ablation and extension bits: accepted on the fast path, rejected on the plain path, and the
    exact ellipse-tile test is rejected together with the extent ablation it refines."""
    ok = ["fast/no-fusion", "fast/exact-tiles", "fast/no-fusion/exact-tiles", "fast/no-key32/exact-tiles",
          "fast/hw-exp2", "fast/hw-exp2/exact-tiles", "fast/no-key32/hw-exp2", "fast/quad-pixel",
          "fast/quad-pixel/exact-tiles", "fast/no-int8sh/quad-pixel", "plain/hw-exp2",
          "fast/" + "/".join("no-" + a for a in B.ABLATIONS)]
    for p in ok:
        assert rgs.workspace_size(1000, 64, 64, p, 4096) > 0
    size = C.c_uint64()
    for word in (B.PATH_FAST | B.ABLATIONS["extent"] | B.EXTENSIONS["exact-tiles"],
                 B.PATH_PLAIN | B.EXTENSIONS["exact-tiles"], B.PATH_PLAIN | B.ABLATIONS["fusion"],
                 B.PATH_FAST | B.ABLATIONS["fastexp"] | B.EXTENSIONS["hw-exp2"],
                 B.PATH_FAST | B.ABLATIONS["dualpixel"] | B.EXTENSIONS["hw-exp2"],
                 B.PATH_PLAIN | B.EXTENSIONS["hw-exp2"] | B.ABLATIONS["fusion"],
                 B.PATH_PLAIN | B.EXTENSIONS["hw-exp2"] | B.EXTENSIONS["exact-tiles"], B.PATH_FAST | (1 << 18), 2,
                 B.PATH_FAST | B.EXTENSIONS["quad-pixel"] | B.EXTENSIONS["hw-exp2"],
                 B.PATH_FAST | B.EXTENSIONS["quad-pixel"] | B.ABLATIONS["fastexp"],
                 B.PATH_FAST | B.EXTENSIONS["quad-pixel"] | B.ABLATIONS["dualpixel"],
                 B.PATH_PLAIN | B.EXTENSIONS["quad-pixel"]):
        assert B.lib.rgs_workspace_size(1000, 64, 64, word, 4096, C.byref(size)) == B.RGS_E_INVALID, hex(word)
    for bad in ("fast/no-nothing", "fast/exact", "plain/exact-tiles", "fast/"):
        with pytest.raises(KeyError):
            B.PATHS[bad]
    # the unfused fast path with exact tiles keeps a 64-bit mask per Gaussian
    assert (rgs.workspace_size(1000, 64, 64, "fast/no-fusion/exact-tiles", 4096)
            >= rgs.workspace_size(1000, 64, 64, "fast/no-fusion", 4096) + 8 * 1000)


def _edge_scene():
    sc = wl.config_scene("small", n=3000)
    sh = sc.sh.copy()
    sh[0] = 0.0                                     # all-zero SH
    sh[1, 1:4, :] = 0.0                             # zero degree-1 blocks
    sh[2, 4:9, 1] = 1e-6                            # subnormal FP16 scale
    sh[3, 9:16, 2] = np.float32(127.0 * 0.25)       # exact ratios
    sh[4, 9, 0] = 1.0
    sh[4, 10, 0] = -1.0 / 254.0                     # q = -0.5 exactly: ties to even
    sh[4, 11, 0] = 3.0 / 254.0                      # q = 1.5
    scales = sc.scales.copy()
    scales[5] = np.float32(1.0 + 2.0 ** -11)        # FP16 midpoint: ties to even
    scales[6] = np.float32(1.0 + 3 * 2.0 ** -11)
    scales[7] = np.float32(3e-8)                    # FP16 subnormal scale
    opa = sc.opacity.copy()
    opa[8] = 1.0
    opa[9] = np.float32(1e-6)
    return wl.Scene(sc.means, scales, sc.quats, opa, sh)


def test_quantize_host_bit_exact_vs_oracle():
    sc = _edge_scene()
    q = rgs.quantize_host(sc)
    fs = oracle.quantize_scene(sc)
    assert np.array_equal(q["quats"], fs.quats.view(np.uint16))
    assert np.array_equal(q["scales"], fs.scales.view(np.uint16))
    assert np.array_equal(q["log_opacity"], fs.log_opacity.view(np.uint16))
    assert np.array_equal(q["sh_q"], fs.sh_q)
    assert np.array_equal(q["sh_scale"], fs.sh_scale.view(np.uint16))


@pytest.mark.parametrize("field,index,value", [
    ("means", (0, 1), np.nan), ("scales", (1, 0), 0.0), ("scales", (1, 2), -1.0),
    ("quats", (2,), 0.0), ("opacity", (3,), 0.0), ("opacity", (3,), 1.5), ("sh", (4, 3, 1), np.inf),
    ("scales", (5, 1), 1e6),
])
def test_quantize_host_rejects(field, index, value):
    sc = wl.config_scene("small", n=50)
    arr = getattr(sc, field).copy()
    arr[index] = value
    setattr(sc, field, arr)
    with pytest.raises(rgs.RGSError) as e:
        rgs.quantize_host(sc)
    assert e.value.status == B.RGS_E_INVALID


def test_no_device_is_reported_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(rgs.RGSError) as e:
        rgs.Context(0)
    assert e.value.status == B.RGS_E_NODEVICE


def test_backward_host_checks_and_scratch_size():
    assert B.lib.rgs_render_backward(None, None, None, 16, 16, None, None, 0, None) == B.RGS_E_INVALID
    assert B.lib.rgs_scene_update_plain(None, None, None) == B.RGS_E_INVALID
    for n, W, H in [(10000, 256, 256), (1000000, 1920, 1080), (5, 17, 33)]:
        ws = rgs.workspace_size(n, W, H, "plain", 4 * n + 65536)
        cap = rgs.workspace_capacity(n, W, H, "plain", ws)
        got = rgs.backward_scratch_size(n, W, H, ws)
        assert got == (cap * 48 + 255) // 256 * 256
    with pytest.raises(rgs.RGSError):
        rgs.backward_scratch_size(100, 64, 64, 1024)          # workspace too small for any entry


def test_null_arguments_are_rejected():
    assert B.lib.rgs_frame_plan(16, 16, None) == B.RGS_E_INVALID
    assert B.lib.rgs_scene_upload(None, None, 1, None) == B.RGS_E_INVALID
    assert B.lib.rgs_render(None, None, None, 16, 16, 0, None, 0, None, None) == B.RGS_E_INVALID
    assert B.lib.rgs_workspace_check(None, None, None, 0) == B.RGS_E_INVALID
    assert B.lib.rgs_ctx_set_timing(None, 1) == B.RGS_E_INVALID
    b = B.C.c_uint64()
    assert B.lib.rgs_render_workspace_bound(None, 1920, 1080, B.PATH_FAST, 0, B.C.byref(b)) == B.RGS_E_INVALID
    assert B.lib.rgs_scene_device_bytes(None, B.C.byref(b)) == B.RGS_E_INVALID


def test_server_config_is_validated_before_device_use():
    def create(**kw):
        cfg = B.ServerConfig(device=0, n_streams=4, mem_budget=1 << 30, use_graphs=1, reserved=0,
                             entries_per_gaussian=0.0)
        for k, v in kw.items():
            setattr(cfg, k, v)
        h = C.c_void_p()
        return B.lib.rgs_server_create(C.byref(cfg), C.byref(h))

    assert create(n_streams=0) == B.RGS_E_INVALID
    assert create(n_streams=17) == B.RGS_E_INVALID
    assert create(mem_budget=0) == B.RGS_E_INVALID
    assert create(entries_per_gaussian=-1.0) == B.RGS_E_INVALID
    assert create(entries_per_gaussian=float("nan")) == B.RGS_E_INVALID
    assert B.lib.rgs_server_create(None, None) == B.RGS_E_INVALID
    import torch
    if not torch.cuda.is_available():
        assert create() == B.RGS_E_NODEVICE
    assert B.lib.rgs_serve(None, None, 0, None, None) == B.RGS_E_INVALID


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's sizes and offsets."""
    structs = {"rgs_camera": B.CameraC, "rgs_frame_stats": B.FrameStats, "rgs_debug_out": B.DebugOut,
               "rgs_plan": B.Plan, "rgs_scene_desc": B.SceneDesc, "rgs_fast_host": B.FastHost,
               "rgs_grads": B.Grads, "rgs_server_config": B.ServerConfig, "rgs_request": B.Request,
               "rgs_response": B.Response, "rgs_server_stats": B.ServerStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rgs.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            s, f, v = ln.split()
            got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
