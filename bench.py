#!/usr/bin/env python3
"""Benchmark of the tile-based 3D Gaussian Splatting forward render on one MI355X.

Default workload (the N=1 line): 1,000,000 seeded Gaussians rendered at
1920x1080 (camera at distance 25, fovx 60 deg).  A step is one frame of the
whole hot path (front end, sort, tile ranges, rasterizer) with the scene
already resident in HBM and the image left on the device.  `value` is the fast
path's frames per second; the plain path's FPS, the speedup, per-frame p50/p99
latency, per-stage times, the dominant kernel's roofline position and the
oracle's CPU rate are reported beside it.  The 3,000,000-Gaussian 3840x2160
64-pose orbit is measured as an extra section (--no-4k skips it).

  python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FPS at 1080p/4K (1M/3M Gaussians) fast vs plain path; p50/p99 latency"

# MI355X peaks.  VALU: 256 CUs x 4 SIMDs, each issuing up to two wave64
# instructions (from two waves) per four cycles onto its 16 lanes, at 2.4 GHz:
# 256 x 4 x 2 x 16 x 2.4e9 = 78.6e12 lane-operations per second, non-packed
# (the published 157.3 TFLOP/s float32 counts an FMA as two).  The dual issue
# is measured, not assumed: the calibration probe (rgs_probe_valu, eight
# independent FMA chains per lane) reaches 0.40 wave instructions per SIMD and
# cycle at eight waves per SIMD, with SQ_ACTIVE_INST_VALU2 counting paired
# issue for 90 % of them (profiles/valu_calibration.txt).  HBM3E 8 TB/s.
VALU_PEAK_TOPS = 256 * 4 * 2 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic VALU lane-operations per blended (pixel, Gaussian) pair -- a pair
# past the skip test that the method must composite.  Fast: the folded exponent
# (5 FMA for the first pixel of a lane, 2 FMA + 1 add for the second: 4 on
# average), the skip test 1, the bit-level exp 2 (FMA + convert), the select 1,
# weight 1, transmittance 1, stop test 1, colour 3.  Plain: offsets 2,
# quadratic 7, exp 2, opacity 1, clamp 1, skip test 1, T (1 - alpha) 2, stop
# test 1, weight 1, colour 3.
OPS_PER_PAIR = {"fast": 14, "plain": 21}
# ... and per blended pair of the backward pass (recomputed alpha, recovered T,
# the nine derivatives and the running colour behind the pair).
OPS_PER_PAIR_BACKWARD = 45

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--orbit-rounds", type=int, default=2)
    ap.add_argument("--no-4k", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-tiles", type=int, default=512, help="tiles the oracle blends (1080p, fast path)")
    ap.add_argument("--cpu-plain-tiles", type=int, default=128, help="of those, tiles the plain oracle blends")
    ap.add_argument("--cpu-4k-poses", default="0,16,32,48")
    ap.add_argument("--cpu-4k-tiles", type=int, default=64, help="tiles the oracle blends per 4K pose")
    ap.add_argument("--cold-frames", type=int, default=50, help="frames of the cold-cache run (0: none)")
    ap.add_argument("--paths", default="fast,plain")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--ablation-steps", type=int, default=100)
    ap.add_argument("--backward-steps", type=int, default=50)
    ap.add_argument("--serve-seconds", type=float, default=1.5, help="schedule length per arrival rate")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device copies of MIB MiB (scale reference for HBM counters)")
    ap.add_argument("--calibrate-valu", action="store_true",
                    help="only run the VALU probe at 1, 2, 4 and 8 waves per SIMD (issue-rate and clock "
                         "reference for the VALU counters)")
    return ap.parse_args()


def stage_bytes(path, n, n_vis, n_dup, n_tiles, passes):
    """Algorithmic HBM bytes per frame of each memory-bound stage.  `path` is
    "plain", "fast", or a fast-path variant "fast/no-<step>/.../<extension>"
    whose removed steps change what is read and written."""
    parts = path.split("/")
    if parts[0] == "plain":
        fe = 44 * n + 192 * n_vis + (48 + 8 + 4) * n_vis + 4 * n
        dup = 4 * n + 12 * n_vis + 12 * n_dup
        kb = 8
    else:
        off = {p[3:] for p in parts[1:] if p.startswith("no-")}
        kb = 8 if "key32" in off else 4
        geom = 12 + (32 if "fp16geom" in off else 16)      # mean + rotation, scale, ln o
        sh = 192 if "int8sh" in off else 72                 # FP32 SH, or INT8 SH + FP16 scales
        fe = geom * n + sh * n_vis + 48 * n_vis
        if "fusion" in off:       # preprocess writes count, rectangle, depth; duplicate reads them
            fe += 4 * n + 12 * n_vis
            dup = 4 * n + 12 * n_vis + (kb + 4) * n_dup
        else:
            fe += (kb + 4) * n_dup
            dup = 0
    sort = passes * 2 * (kb + 4) * n_dup          # Eq. sort_memory: read + write per pass
    ranges = kb * n_dup + 8 * n_tiles
    return dict(frontend=fe, duplicate=dup, sort=sort, ranges=ranges)


def ops_per_pair(path):
    """Algorithmic lane-ops per blended pair of a path or fast-path variant (an
    exponential counts 2, as in Eq. fma_exp or a scale and an exp2)."""
    if path == "plain":
        return OPS_PER_PAIR["plain"]
    return OPS_PER_PAIR["fast"] + (1 if "no-dualpixel" in path.split("/") else 0)


def kernel_sha(name):
    with open(os.path.join(ROOT, "paper_2608_15785_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_counters(kernel, workload, src):
    """The committed rocprofv3 counter record of a kernel (HBM bytes and VALU
    wave instructions per launch), if it was taken on the current source of
    the kernel; else {}."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if not line.startswith("{"):
            continue
        rec = json.loads(line)
        if "<true" in rec.get("instance", ""):       # a counting (debug) render's launch
            continue
        if rec.get("kernel") == kernel and rec.get("workload") == workload and \
                rec.get("source_sha") == kernel_sha(src):
            return rec
    return {}


def measured_traffic(kernel, workload, src):
    """HBM bytes per launch from the committed counter summary, or None."""
    return measured_counters(kernel, workload, src).get("bytes_per_launch")


def time_path(R, ds, cams, path, steps, warmup, lat_frames):
    """Throughput over `steps` frames cycling through `cams` (nothing but the
    frames on the stream), then the same number of frames with the library's
    per-stage HIP events on its stream (each recorded event idles the GPU for a
    few microseconds, so they stay out of the throughput loop), then per-frame
    latency between events bracketing back-to-back frames."""
    import torch
    W, H = cams[0].width, cams[0].height
    need = 0
    for cam in cams:                       # size the workspace for every pose (synchronous)
        _, st = R.render(ds, cam, path)
        need = max(need, st["n_entries"])
    R.workspace(ds.n, W, H, path, int(need * 1.05) + 4096)
    for k in range(warmup):
        R.render(ds, cams[k % len(cams)], path, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        R.render(ds, cams[k % len(cams)], path, check=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    chk = R.check(ds, cams[(steps - 1) % len(cams)], path)
    assert chk["overflow"] == 0 and chk["device_error"] == 0, chk
    R.ctx.set_timing(True)
    for k in range(steps):
        R.render(ds, cams[k % len(cams)], path, check=False)
    stage_ms, nf = R.ctx.collect_timing()
    R.ctx.set_timing(False)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(lat_frames)]
    for k in range(lat_frames):
        ev[k][0].record()
        R.render(ds, cams[k % len(cams)], path, check=False)
        ev[k][1].record()
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    sec = (t1 - t0) / steps
    return dict(fps=1.0 / sec, ms_per_frame=sec * 1e3,
                stage_ms={k: v / max(nf, 1) for k, v in stage_ms.items()},
                latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                                mean=float(lat.mean())))


def pixels_per_lane(path):
    parts = path.split("/")
    if parts[0] == "plain":
        return 1
    return 4 if "quad-pixel" in parts else (1 if "no-dualpixel" in parts else 2)


def frame_counts(R, ds, cam, path):
    """Entry and pair counts of one frame from a counting render: pairs visited up to each
    pixel's stop, pairs blended, and (fast path) pairs evaluated by the rasterizer's waves:
    every list entry a wave evaluates is evaluated at all of its 64 x pixels-per-lane pixels."""
    g = R.render_debug(ds, cam, path)
    st = g["stats"]
    c = dict(n_visible=int(st["n_visible"]), n_entries=int(st["n_entries"]),
             pairs_visited=int(g["n_proc"].astype(np.int64).sum()),
             pairs=int(g["n_blend"].astype(np.int64).sum()), passes=int(st["passes"]))
    if path != "plain":
        c["list_steps"] = int(st["list_steps"])
        c["pairs_evaluated"] = int(st["list_steps"]) * 64 * pixels_per_lane(path)
    return c


def bucket_sorted(path, n_tiles):
    """Whether the library sorts this frame's keys with the bucket sort (the top-digit radix
    pass, then the other three digits per bucket in LDS, which also writes the tile ranges):
    the fast path's 32-bit keys with 2^8 .. 2^14 tiles."""
    b_t = max(1, int(np.ceil(np.log2(n_tiles))))
    return path.split("/")[0] == "fast" and "no-key32" not in path.split("/") and 8 <= b_t <= 14


def rooflines(path, counts, stage_ms, n, n_tiles):
    by = stage_bytes(path, n, counts["n_visible"], counts["n_entries"], n_tiles, counts["passes"])
    bucket = bucket_sorted(path, n_tiles)
    if bucket:
        # the ranges stage holds only the rasterizers' schedule (read 8 B, write 4 B per tile)
        by["ranges"] = 12 * n_tiles
    out = {}
    for s, b in by.items():
        ms = stage_ms.get(s, 0.0)
        if b and ms > 0:
            gbs = b / (ms * 1e-3) / 1e9
            out[s] = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=round(gbs / HBM_PEAK_GBS, 4), bytes=int(b), ms=round(ms, 4))
    if "sort" in out:
        # Eq. sort_memory counts every pass; the bucket sort moves keys and values through
        # HBM twice (the top-digit pass, then each bucket once) for the same four digits
        out["sort"]["hbm_passes"] = 2 if bucket else counts["passes"]
    ms = stage_ms["raster"]
    ops = ops_per_pair(path)
    tops = counts["pairs"] * ops / (ms * 1e-3) / 1e12
    out["raster"] = dict(bound="alu", achieved=round(tops, 3), peak=round(VALU_PEAK_TOPS, 2),
                         unit="Tops/s", frac=round(tops / VALU_PEAK_TOPS, 4), pairs_blended=counts["pairs"],
                         pairs_visited=counts["pairs_visited"], ops_per_pair=ops, ms=round(ms, 4))
    if counts.get("pairs_evaluated"):
        out["raster"]["pairs_evaluated"] = counts["pairs_evaluated"]
        out["raster"]["evaluated_per_blended"] = round(counts["pairs_evaluated"] / max(counts["pairs"], 1), 3)
    return out


PROBE_ITERS = 20000


def calibrate_valu(rgs, torch):
    """The VALU probe (8 * PROBE_ITERS FMA instructions per wave) at 1, 2, 4
    and 8 waves per SIMD, each dispatch timed with events on its stream; a
    profiler run of this mode reads the same dispatches' VALU and cycle
    counters."""
    from paper_2608_15785_amd import _binding as B
    R = rgs.Renderer(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = []
    for waves_per_simd in (1, 2, 4, 8):
        blocks = cus * waves_per_simd          # 256-thread workgroups: 4 waves, one per SIMD
        buf = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
        for rep in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            B.probe_valu(R.ctx, blocks, PROBE_ITERS, buf)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
        waves = blocks * 4
        insts = waves * 8 * PROBE_ITERS
        out.append({"waves_per_simd": waves_per_simd, "blocks": blocks, "ms": round(ms, 4),
                    "fma_wave_insts": insts,
                    "insts_per_simd_cycle_at_2.4GHz": round(insts / (ms * 1e-3 * cus * 4 * 2.4e9), 4)})
        del buf
    return {"calibrate_valu": out, "iters": PROBE_ITERS, "cus": cus}


def _oracle_frame_rate(oracle, arr, cam, path, n_tiles_sample, seed, cores):
    """One frame of the FP64 oracle on the host: front end, keys and sort of all Gaussians
    (one core), then blending of a seeded sample of tiles on `cores` processes.  Returns the
    time scaled to the full frame and the sampled frame (its images cover the sample)."""
    modes = ("fast-def", "fast-exact") if path == "fast" else ("plain",)
    t = time.perf_counter()
    fr = oracle.render(arr, cam, path, modes=modes, blend=False)
    t_front = time.perf_counter() - t
    n_t = fr.plan.n_tiles
    k = min(n_tiles_sample, n_t)
    tiles = np.random.default_rng(seed).choice(n_t, k, replace=False)
    t = time.perf_counter()
    fr = oracle.render(arr, cam, path, modes=modes, tiles=tiles, workers=cores)
    t_blend = max(time.perf_counter() - t - t_front, 0.0)
    return t_front, t_blend, k, n_t, fr


def _tile_mask(fr):
    m = np.zeros((fr.plan.height, fr.plan.width), bool)
    for t in fr.tiles:
        tx, ty = int(t) % fr.plan.tiles_x, int(t) // fr.plan.tiles_x
        m[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = True
    return m


def _psnr(a, b, mask):
    d = (a - b)[:, mask]
    mse = float(np.mean(d * d))
    return None if mse == 0 else round(10 * math.log10(1.0 / mse), 3)


def cpu_baseline(R, ds, scene, cam, n_tiles_sample, plain_tiles):
    """The FP64 oracle on the host cores (the CPU baseline), and the accuracy of the GPU
    images measured against the oracle frames it renders: PSNR (peak 1, unclipped values)
    over the oracle's sampled tiles of the fast GPU image against the bit-level-exp and
    exact-exp oracles, of the plain GPU image against the plain oracle, and the
    quantisation loss: the fast GPU image against the plain oracle on the FP32 scene."""
    import torch
    import oracle
    cores = min(16, os.cpu_count() or 1)
    fast_arr = oracle.prepare_fast(oracle.quantize_scene(scene))
    t_front, t_blend, k, n_t, fr = _oracle_frame_rate(oracle, fast_arr, cam, "fast", n_tiles_sample, 0, cores)
    frame_s = t_front + t_blend * n_t / k
    base = dict(value=round(1.0 / frame_s, 5), unit="FPS", cores=cores, kind="oracle",
                sample=f"FP64 oracle, fast path, {scene.n} Gaussians at {cam.width}x{cam.height}: front end, "
                       f"keys and sort of all Gaussians ({t_front:.1f} s, one core) plus blending of {k} of "
                       f"{n_t} seeded tiles on {cores} processes ({t_blend:.1f} s), scaled to the full frame "
                       f"({frame_s:.1f} s per frame)")
    img_fast = R.render(ds, cam, "fast")[0].cpu().numpy().astype(np.float64)
    img_plain = R.render(ds, cam, "plain")[0].cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    m = _tile_mask(fr)
    plain_arr = oracle.prepare_plain(scene)
    plain_sample = fr.tiles[:plain_tiles]
    frp = oracle.render(plain_arr, cam, "plain", tiles=plain_sample, workers=cores)
    mp = _tile_mask(frp)
    acc = {"tiles_fast": int(k), "tiles_plain": int(len(plain_sample)),
           "fast_vs_oracle_bitexp": _psnr(img_fast, fr.images["fast-def"], m),
           "fast_vs_oracle_exactexp": _psnr(img_fast, fr.images["fast-exact"], m),
           "plain_vs_oracle": _psnr(img_plain, frp.images["plain"], mp),
           "quantisation_loss_fast_vs_plain_oracle": _psnr(img_fast, frp.images["plain"], mp),
           "oracle_fast_vs_oracle_plain": _psnr(fr.images["fast-def"], frp.images["plain"], mp),
           "note": "None = identical; peak 1.0"}
    return base, acc


def cpu_baseline_4k(R, ds, scene, poses, n_tiles_sample):
    """The FP64 oracle's fast path at 3840x2160 on orbit poses (front end of all 3M
    Gaussians on one core, blending of a tile sample on the host's processes, scaled to
    the frame), and the fast GPU image's PSNR against it on those tiles."""
    import torch
    import oracle
    import workloads as wl
    cores = min(16, os.cpu_count() or 1)
    arr = oracle.prepare_fast(oracle.quantize_scene(scene))
    per_pose = {}
    for pose in poses:
        cam = wl.config_camera("4k", pose=pose)
        t_front, t_blend, k, n_t, fr = _oracle_frame_rate(oracle, arr, cam, "fast", n_tiles_sample, 100 + pose,
                                                          cores)
        frame_s = t_front + t_blend * n_t / k
        img = R.render(ds, cam, "fast")[0].cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        m = _tile_mask(fr)
        per_pose[str(pose)] = {"s_per_frame": round(frame_s, 2), "front_s": round(t_front, 2),
                               "blend_s_sample": round(t_blend, 2), "tiles": int(k),
                               "psnr_fast_vs_oracle_bitexp": _psnr(img, fr.images["fast-def"], m),
                               "psnr_fast_vs_oracle_exactexp": _psnr(img, fr.images["fast-exact"], m)}
        log(f"[bench] cpu baseline 4k pose {pose}: {per_pose[str(pose)]}")
    mean_s = float(np.mean([v["s_per_frame"] for v in per_pose.values()]))
    return {"value": round(1.0 / mean_s, 5), "unit": "FPS", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, fast path, 3,000,000 Gaussians at 3840x2160, orbit poses {list(poses)}: "
                      f"front end, keys and sort of all Gaussians on one core plus blending of {n_tiles_sample} "
                      f"seeded tiles per pose on {cores} processes, scaled to the frame",
            "poses": per_pose}


def serving_section(rgs, wl, torch, dev_scenes, args):
    """Poisson request schedules at 200/500/1000 req/s over the two resident scenes,
    resolutions 50% 720p / 35% 1080p / 15% 4K, fast path through graph replays."""
    res_list = [(1280, 720), (1920, 1080), (3840, 2160)]
    ring = {wh: [torch.empty((3, wh[1], wh[0]), dtype=torch.float32, device="cuda") for _ in range(8)]
            for wh in res_list}
    torch.cuda.synchronize()

    def schedule(rate, n, seed, burst_all=False):
        arr, res, sc, pose = wl.poisson_requests(rate, n, seed=seed)
        arr = np.zeros(n) if burst_all else arr - arr[0]
        reqs = []
        for i in range(n):
            wh = (int(res[i][0]), int(res[i][1]))
            cam = wl.serving_camera(int(sc[i]), int(pose[i]), *wh)
            reqs.append((dev_scenes[int(sc[i])], cam, "fast", float(arr[i]), ring[wh][i % 8]))
        return reqs

    def summarise(resp, st, n):
        lat = np.array([r["latency"] for r in resp if r["status"] == 0]) * 1e3
        ok = int(np.sum([r["status"] == 0 for r in resp]))
        return {"requests": n, "ok": ok, "retried": int(sum(r["retried"] for r in resp)),
                "fps": round(ok / st["wall"], 1) if st["wall"] > 0 else None,
                "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                               "p99": round(float(np.percentile(lat, 99)), 4),
                               "mean": round(float(lat.mean()), 4)},
                "max_in_flight": st["max_in_flight"], "mean_in_flight": round(st["mean_in_flight"], 3),
                "ws_gib_peak": round(st["ws_bytes_peak"] / 2**30, 2), "n_evicted": st["n_evicted"]}

    budget = 32 << 30
    out = {"n_streams": args.serve_streams, "mem_budget_gib": budget >> 30, "graphs": True,
           "mix": "50% 1280x720, 35% 1920x1080, 15% 3840x2160; scenes 1M / 3M equally; random orbit pose"}
    srv = rgs.Server(0, n_streams=args.serve_streams, mem_budget=budget, use_graphs=True,
                     entries_per_gaussian=6.0)
    # warm-up: every class once per slot, so workspaces and graphs exist before timing
    warm = []
    for s_idx in range(2):
        for wh in res_list:
            for k in range(args.serve_streams):
                cam = wl.serving_camera(s_idx, 5 * k, *wh)
                warm.append((dev_scenes[s_idx], cam, "fast", 0.0, ring[wh][k]))
    _, st = srv.serve(warm)
    srv.serve(warm)
    out["warmup"] = {"requests": len(warm), "graphs_captured": st["n_captured"],
                     "ws_gib": round(st["ws_bytes_held"] / 2**30, 2)}
    rates = {}
    for rate in (200, 500, 1000):
        n = max(50, int(rate * args.serve_seconds))
        resp, st = srv.serve(schedule(rate, n, 3))
        rates[str(rate)] = summarise(resp, st, n)
        log(f"[bench] serving {rate} req/s: {rates[str(rate)]}")
    out["rates"] = rates
    n_sat = 600
    resp, st = srv.serve(schedule(1000, n_sat, 7, burst_all=True))
    out["saturation"] = summarise(resp, st, n_sat)
    log(f"[bench] serving saturation: {out['saturation']}")
    srv.close()
    for label, streams, graphs in (("saturation_direct_launch", args.serve_streams, False),
                                   ("saturation_one_stream", 1, True)):
        s2 = rgs.Server(0, n_streams=streams, mem_budget=budget, use_graphs=graphs, entries_per_gaussian=6.0)
        s2.serve(warm)
        resp, st = s2.serve(schedule(1000, n_sat, 7, burst_all=True))
        out[label] = summarise(resp, st, n_sat)
        log(f"[bench] serving {label}: {out[label]}")
        s2.close()
    del ring
    return out


def cold_cache_section(torch, R, ds, cam, path, frames, n, n_tiles):
    """Frames of `path` each preceded by a 1 GiB device write, which evicts the scene and
    the frame's transients from the 256 MB Infinity Cache: per-stage times from the
    library's stage events (the writes lie outside them) and the stages' roofline
    fractions against the same algorithmic bytes as the warm frames."""
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    R.render(ds, cam, path)
    R.ctx.set_timing(True)
    for k in range(frames):
        flush.fill_(float(k))
        R.render(ds, cam, path, check=False)
    stage_ms, nf = R.ctx.collect_timing()
    R.ctx.set_timing(False)
    torch.cuda.synchronize()
    del flush
    stage_ms = {k: v / max(nf, 1) for k, v in stage_ms.items()}
    c = frame_counts(R, ds, cam, path)
    rl = rooflines(path, c, stage_ms, n, n_tiles)
    return {"frames": nf, "flush_bytes": 1 << 30, "ms_per_frame": round(sum(stage_ms.values()), 4),
            "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
            "roofline_frac": {k: v["frac"] for k, v in rl.items()}}


ABLATIONS = ["fastexp", "dualpixel", "fusion", "extent", "key32", "int8sh", "fp16geom"]


def ablation_section(R, ds, cam, steps, n_tiles):
    """The fast path with each of Sec. IV's optimisations removed in turn (and
    all of them), and with each extension (the exact ellipse-tile test, the
    hardware exp2) added, on the 1M/1080p workload: FPS, stage times, entries,
    passes."""
    out = {}
    paths = ["fast"] + ["fast/no-" + a for a in ABLATIONS] + ["fast/" + "/".join("no-" + a for a in ABLATIONS),
                                                              "plain", "fast/exact-tiles", "fast/hw-exp2",
                                                              "fast/quad-pixel"]
    for path in paths:
        r = time_path(R, ds, [cam], path, steps, 10, 20)
        c = frame_counts(R, ds, cam, path)
        name = "all" if path.count("/") > 1 else path.replace("fast/no-", "no-").replace("fast/", "+")
        rl = rooflines(path, c, r["stage_ms"], ds.n, n_tiles)
        out[name] = {"fps": round(r["fps"], 1), "ms_per_frame": round(r["ms_per_frame"], 4),
                     "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items()},
                     "n_entries": c["n_entries"], "passes": c["passes"], "pairs_visited": c["pairs_visited"],
                     "pairs_evaluated": c.get("pairs_evaluated"),
                     "roofline_frac": {k: v["frac"] for k, v in rl.items()}}
        log(f"[bench] ablation {path}: {out[name]['fps']} FPS, stages {out[name]['stage_ms']}")
    base = out["fast"]["fps"]
    for k, v in out.items():
        v["fps_vs_fast"] = round(v["fps"] / base, 3)
    return out


def differentiation_section(rgs, wl, torch, R, sc, cam, steps, warmup, path="plain"):
    """One training step at 1M Gaussians, 1920x1080: write the parameters into the
    device scene, render the plain path (or its training variant "plain/hw-exp2",
    whose forward and backward take exp through the hardware exp2), L1 loss
    gradient against a render of the scene with means perturbed by N(0, 0.01),
    backward to the activated parameters."""
    from paper_2608_15785_amd import _binding as B
    W, H = cam.width, cam.height
    dev = "cuda"
    tgt_scene = wl.Scene(means=wl.perturbed_means(sc), scales=sc.scales, quats=sc.quats, opacity=sc.opacity,
                         sh=sc.sh)
    dt = R.upload(tgt_scene, ("plain",))
    target, _ = R.render(dt, cam, "plain")
    target = target.clone()
    dt.release()
    ds = R.upload(sc, ("plain",))
    params = [torch.tensor(np.ascontiguousarray(a, np.float32), device=dev)
              for a in (sc.means, sc.scales, sc.quats, sc.opacity, sc.sh)]
    _, st = R.render(ds, cam, path)
    ws = R.workspace(sc.n, W, H, path, int(st["n_entries"] * 1.05) + 4096)
    out = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    scratch = torch.empty(rgs.backward_scratch_size(sc.n, W, H, ws.numel()), dtype=torch.uint8, device=dev)
    inv_n = 1.0 / out.numel()
    ev = {k: torch.cuda.Event(enable_timing=True) for k in ("a", "b", "c", "d", "e")}

    def step(timed=False):
        if timed:
            ev["a"].record()
        rgs.scene_update_plain(R.ctx, ds, *params)
        if timed:
            ev["b"].record()
        B.render(R.ctx, ds, cam, path, ws, out)
        if timed:
            ev["c"].record()
        dimg = torch.sign(out - target) * inv_n
        if timed:
            ev["d"].record()
        g = rgs.render_backward(R.ctx, ds, cam, ws, dimg, scratch=scratch)
        if timed:
            ev["e"].record()
        return g

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    chk = rgs.workspace_check(R.ctx, ws, sc.n)
    assert chk["overflow"] == 0 and chk["device_error"] == 0, chk
    parts = {"update": 0.0, "forward": 0.0, "loss_grad": 0.0, "backward": 0.0}
    for _ in range(steps):
        step(timed=True)
        torch.cuda.synchronize()
        parts["update"] += ev["a"].elapsed_time(ev["b"])
        parts["forward"] += ev["b"].elapsed_time(ev["c"])
        parts["loss_grad"] += ev["c"].elapsed_time(ev["d"])
        parts["backward"] += ev["d"].elapsed_time(ev["e"])
    parts = {k: round(v / steps, 4) for k, v in parts.items()}
    dbg = R.render_debug(ds, cam, path)
    pairs = int(dbg["n_blend"].astype(np.int64).sum())
    loss = float((out - target).abs().mean())
    ds.release()
    bwd_s = parts["backward"] * 1e-3
    achieved = pairs * OPS_PER_PAIR_BACKWARD / bwd_s / 1e12
    return {"workload": f"training: 1,000,000 Gaussians, 1920x1080, {path} path, L1 loss against a render with "
                        "means + N(0, 0.01)",
            "steps": steps, "ms_per_step": round((t1 - t0) / steps * 1e3, 4),
            "steps_per_s": round(steps / (t1 - t0), 2), "stage_ms": parts, "l1_loss": loss,
            "pairs_blended": pairs,
            "roofline_backward": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                                  "unit": "T lane-op/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                                  "ops_per_pair": OPS_PER_PAIR_BACKWARD,
                                  "note": "whole backward call (both kernels and the header read)"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the renderer runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2608_15785_amd as rgs
    import workloads as wl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 5}))
        return
    if args.calibrate_valu:
        print(json.dumps(calibrate_valu(rgs, torch)), flush=True)
        return
    paths = [p for p in args.paths.split(",") if p]
    R = rgs.Renderer(0)

    log("[bench] 1080p: 1,000,000 Gaussians, 1920x1080")
    sc1 = wl.config_scene("1080p")
    cam1 = wl.config_camera("1080p")
    ds1 = R.upload(sc1)
    plan1 = rgs.frame_plan(cam1.width, cam1.height)
    res1 = {}
    for path in paths:
        r = time_path(R, ds1, [cam1], path, args.steps, args.warmup, args.latency_frames)
        r.update(frame_counts(R, ds1, cam1, path))
        r["roofline"] = rooflines(path, r, r["stage_ms"], sc1.n, plan1["n_tiles"])
        res1[path] = r
        log(f"[bench] 1080p {path}: {r['fps']:.1f} FPS, stages {r['stage_ms']}")

    cold = {}
    if args.cold_frames > 0:
        for path in paths:
            cold[path] = cold_cache_section(torch, R, ds1, cam1, path, args.cold_frames, sc1.n, plan1["n_tiles"])
            log(f"[bench] 1080p {path} cold cache: {cold[path]}")

    cpu, accuracy = None, None
    if not args.no_cpu_baseline and "fast" in paths and "plain" in paths:
        log("[bench] cpu baseline (oracle) and accuracy against it")
        cpu, accuracy = cpu_baseline(R, ds1, sc1, cam1, args.cpu_tiles, args.cpu_plain_tiles)
        log(f"[bench] accuracy: {accuracy}")

    ablation = None
    if not args.no_ablation and "fast" in paths:
        log("[bench] ablation: the fast path without each optimisation, 1M Gaussians at 1080p")
        ablation = ablation_section(R, ds1, cam1, args.ablation_steps, plan1["n_tiles"])

    diff = None
    if not args.no_backward:
        log("[bench] differentiation: forward + backward, 1M Gaussians at 1080p")
        diff = differentiation_section(rgs, wl, torch, R, sc1, cam1, args.backward_steps, 5)
        log(f"[bench] differentiation: {diff['ms_per_step']} ms/step, stages {diff['stage_ms']}")
        diff["hw_exp2_variant"] = differentiation_section(rgs, wl, torch, R, sc1, cam1, args.backward_steps, 5,
                                                          path="plain/hw-exp2")
        log(f"[bench] differentiation (plain/hw-exp2): {diff['hw_exp2_variant']['ms_per_step']} ms/step, "
            f"stages {diff['hw_exp2_variant']['stage_ms']}")

    res2 = {}
    cpu4k = None
    if not args.no_4k:
        log("[bench] 4k: 3,000,000 Gaussians, 3840x2160, 64-pose orbit")
        ds1.release()
        sc2 = wl.config_scene("4k")
        cams = [wl.config_camera("4k", pose=k) for k in range(64)]
        ds2 = R.upload(sc2)
        plan2 = rgs.frame_plan(3840, 2160)
        for path in paths:
            r = time_path(R, ds2, cams, path, 64 * args.orbit_rounds, 64, 128)
            r.update(frame_counts(R, ds2, cams[0], path))
            r["roofline_pose0"] = rooflines(path, r, r["stage_ms"], sc2.n, plan2["n_tiles"])
            res2[path] = r
            log(f"[bench] 4k {path}: {r['fps']:.1f} FPS, stages {r['stage_ms']}")
        if not args.no_cpu_baseline and "fast" in paths:
            poses = [int(p) for p in args.cpu_4k_poses.split(",") if p]
            cpu4k = cpu_baseline_4k(R, ds2, sc2, poses, args.cpu_4k_tiles)
        if args.no_serving:
            ds2.release()

    serving = None
    if not args.no_serving:
        log("[bench] serving: 1M and 3M scenes resident, Poisson arrivals")
        if args.no_4k:
            sc2 = wl.config_scene("4k")
            ds2 = R.upload(sc2, ("fast",))
        ds1b = R.upload(sc1, ("fast",))
        try:
            serving = serving_section(rgs, wl, torch, [ds1b, ds2], args)
        except rgs.RGSError as e:
            serving = {"error": str(e)}
            log(f"[bench] serving failed: {e}")
        ds1b.release()
        ds2.release()

    main_path = "fast" if "fast" in res1 else paths[0]
    m = res1[main_path]
    stages = {k: v for k, v in m["roofline"].items()}
    dom = max(stages, key=lambda s: stages[s]["ms"])
    kernel = {"raster": "k_raster_fast" if main_path == "fast" else "k_raster_plain",
              "frontend": "k_frontend_fast" if main_path == "fast" else "k_preprocess_plain",
              "duplicate": "k_duplicate", "sort": "k_radix_pass", "ranges": "k_ranges"}[dom]
    src = {"raster": "k_raster.hip", "frontend": "k_frontend.hip", "duplicate": "k_frontend.hip",
           "sort": "k_sort.hip", "ranges": "k_sort.hip"}[dom]
    rl = dict(stages[dom])
    counters = measured_counters(kernel, "1080p-" + main_path, src)
    roofline = {"bound": rl["bound"], "achieved": rl["achieved"], "peak": rl["peak"], "unit": rl["unit"],
                "frac": rl["frac"], "traffic": counters.get("bytes_per_launch"),
                "kernel": kernel, "stage_ms": rl["ms"]}
    for k in ("pairs_blended", "pairs_evaluated", "evaluated_per_blended", "ops_per_pair"):
        if k in rl:
            roofline[k] = rl[k]
    if rl["unit"] == "Tops/s":
        # the same figure against one wave64 instruction per SIMD per four cycles (no dual
        # issue): 39.3 T lane-ops/s, half the peak above
        roofline["frac_single_issue_peak"] = round(rl["achieved"] / (VALU_PEAK_TOPS / 2), 4)
    if counters.get("valu_wave_insts"):
        # from the profiling run that counted them (profiles/traffic_counters.txt): VALU wave
        # instructions per launch (SQ_INSTS_VALU), the launch's duration and the clock
        # (GRBM_GUI_ACTIVE over the duration, per XCD) in that same run, and the issue rate they
        # give per SIMD and cycle (the dual-issue ceiling is 0.5)
        for k in ("valu_wave_insts", "valu_run_duration_us", "valu_run_clock_ghz", "valu_insts_per_simd_cycle",
                  "valu_dual_issue_share", "lds_insts"):
            if k in counters:
                roofline[k] = counters[k]
        if rl.get("pairs_evaluated"):
            roofline["valu_lane_ops_per_evaluated_pair"] = round(
                counters["valu_wave_insts"] * 64 / rl["pairs_evaluated"], 2)

    out = {
        "metric": METRIC,
        "value": round(m["fps"], 2),
        "unit": "FPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_frame"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"1080p: 1,000,000 seeded Gaussians, 1920x1080, {main_path} path "
                               "(INT8 SH + FP16 geometry, 32-bit key, fused front end, dual-pixel, "
                               "bit-level exp)" if main_path == "fast" else
                               "1080p: 1,000,000 seeded Gaussians, 1920x1080, plain path",
                   "n_gaussians": sc1.n, "width": 1920, "height": 1080, "path": main_path},
        "roofline": roofline,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if cpu4k is not None:
        out["cpu_baseline_4k"] = cpu4k
    if accuracy is not None:
        out["psnr"] = {"1080p": accuracy}
        if cpu4k is not None:
            out["psnr"]["4k"] = {p: {k: v for k, v in r.items() if k.startswith("psnr")}
                                 for p, r in cpu4k["poses"].items()}
    out["latency_ms"] = m["latency_ms"]
    out["paths_1080p"] = {p: {k: r.get(k) for k in ("fps", "ms_per_frame", "latency_ms", "stage_ms", "n_visible",
                                                      "n_entries", "pairs", "pairs_visited", "pairs_evaluated",
                                                      "list_steps", "passes", "roofline")}
                          for p, r in res1.items()}
    if cold:
        out["cold_cache_1080p"] = cold
    if "fast" in res1 and "plain" in res1:
        out["speedup_fast_over_plain_1080p"] = round(res1["fast"]["fps"] / res1["plain"]["fps"], 3)
    if ablation is not None and "all" in ablation:
        out["speedup_fast_over_all_seven_removed_1080p"] = round(ablation["fast"]["fps"] / ablation["all"]["fps"],
                                                                 3)
    if res2:
        out["paths_4k_orbit"] = {p: {k: r.get(k) for k in ("fps", "ms_per_frame", "latency_ms", "stage_ms",
                                                             "n_visible", "n_entries", "pairs", "pairs_visited",
                                                             "pairs_evaluated", "passes", "roofline_pose0")}
                                 for p, r in res2.items()}
        if "fast" in res2 and "plain" in res2:
            out["speedup_fast_over_plain_4k"] = round(res2["fast"]["fps"] / res2["plain"]["fps"], 3)
    if serving is not None:
        out["serving"] = serving
    if diff is not None:
        out["differentiation"] = diff
    if ablation is not None:
        out["ablation_1080p"] = ablation
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
