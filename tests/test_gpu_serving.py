"""Request server (continuous batching, graph replay) through the C ABI (needs an MI355X).

Every served image must equal, bit for bit, the image rgs_render gives for the
same request alone; one small request is also checked against the oracle.
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import workloads as wl
from parity import compare_image, oracle_frame

pytestmark = pytest.mark.gpu

RES = [(1280, 720), (1920, 1080), (3840, 2160)]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_15785_amd as rgs
    R = rgs.Renderer(0)
    scenes = [wl.config_scene("1080p", n=200_000), wl.config_scene("4k", n=300_000)]
    small = wl.config_scene("small")
    dev = [R.upload(s) for s in scenes]
    dsmall = R.upload(small)
    return dict(rgs=rgs, R=R, scenes=scenes, dev=dev, small=small, dsmall=dsmall, torch=torch)


def schedule(env, n, rate, burst, plain_every=0, seed=3):
    """Poisson arrivals with the serving resolution mix over the two resident scenes;
    the first ``burst`` requests arrive together so that frames overlap."""
    torch = env["torch"]
    arr, res, sc, pose = wl.poisson_requests(rate, n, seed=seed)
    arr = arr - arr[0]
    arr[:burst] = 0.0
    reqs = []
    for i in range(n):
        W, H = (int(v) for v in res[i])
        cam = wl.serving_camera(int(sc[i]), int(pose[i]), W, H)
        path = "plain" if plain_every and i % plain_every == plain_every - 1 else "fast"
        out = torch.full((3, H, W), float("nan"), dtype=torch.float32, device="cuda:0")
        reqs.append((env["dev"][int(sc[i])], cam, path, float(arr[i]), out))
    return reqs


def alone(env, req):
    ds, cam, path, _, _ = req
    img, st = env["R"].render(ds, cam, path)
    env["torch"].cuda.synchronize()
    return img


def assert_same_as_alone(env, reqs, resp):
    torch = env["torch"]
    torch.cuda.synchronize()
    for i, (req, rp) in enumerate(zip(reqs, resp)):
        assert rp["status"] == 0, (i, rp)
        ref = alone(env, req)
        out = req[4]
        same = torch.equal(out, ref)
        if not same:
            d = (out - ref).abs().max().item()
            raise AssertionError(f"request {i} ({req[1].width}x{req[1].height} {req[2]}): served image differs "
                                 f"from the image rendered alone by up to {d}")


def test_mixed_schedule_matches_alone_and_replays(env):
    rgs = env["rgs"]
    reqs = schedule(env, 24, rate=1000.0, burst=6, plain_every=5)
    _log(f"[serve] graphs: 24 requests, classes {len({(id(r[0]), r[1].width, r[2]) for r in reqs})}")
    srv = rgs.Server(0, n_streams=4, mem_budget=24 << 30, use_graphs=True, entries_per_gaussian=12.0)
    resp, st = srv.serve(reqs)
    _log(f"[serve] stats {st}")
    assert all(r["graph"] == 1 for r in resp)
    assert st["max_in_flight"] >= 2, "frames of the burst did not overlap"
    assert st["n_captured"] >= 1
    assert_same_as_alone(env, reqs, resp)
    # replay the captured graphs once more, with eager renders done in between
    for r in reqs:
        r[4].fill_(float("nan"))
    resp2, st2 = srv.serve(reqs)
    _log(f"[serve] second pass stats {st2}")
    assert st2["n_captured"] == 0, "graphs were captured again"
    assert_same_as_alone(env, reqs, resp2)
    srv.close()


def test_launches_without_graphs_give_the_same_images(env):
    rgs, torch = env["rgs"], env["torch"]
    reqs = schedule(env, 12, rate=2000.0, burst=4, seed=5)
    _log("[serve] graphs vs direct launches, 12 requests")
    a = rgs.Server(0, n_streams=3, mem_budget=24 << 30, use_graphs=True, entries_per_gaussian=12.0)
    resp_a, _ = a.serve(reqs)
    torch.cuda.synchronize()
    first = [r[4].clone() for r in reqs]
    a.close()
    for r in reqs:
        r[4].fill_(float("nan"))
    b = rgs.Server(0, n_streams=3, mem_budget=24 << 30, use_graphs=False, entries_per_gaussian=12.0)
    resp_b, st_b = b.serve(reqs)
    torch.cuda.synchronize()
    assert all(r["graph"] == 0 for r in resp_b) and st_b["n_captured"] == 0
    for i, r in enumerate(reqs):
        assert resp_a[i]["status"] == 0 and resp_b[i]["status"] == 0
        assert torch.equal(first[i], r[4]), i
    b.close()


def test_overflow_is_rendered_again_and_the_class_grows(env):
    rgs, torch = env["rgs"], env["torch"]
    ds = env["dev"][0]
    cam = wl.serving_camera(0, 7, 1920, 1080)
    reqs = []
    for k in range(3):      # far apart: each starts after the previous finished
        out = torch.full((3, 1080, 1920), float("nan"), dtype=torch.float32, device="cuda:0")
        reqs.append((ds, cam, "fast", 0.05 * k, out))
    _log("[serve] overflow: 3 requests with a 65536-entry first workspace")
    srv = rgs.Server(0, n_streams=2, mem_budget=8 << 30, use_graphs=True, entries_per_gaussian=0.01)
    resp, st = srv.serve(reqs)
    _log(f"[serve] {resp} {st}")
    assert resp[0]["retried"] == 1 and resp[0]["n_entries"] > 65536
    assert resp[1]["retried"] == 0 and resp[2]["retried"] == 0
    assert_same_as_alone(env, reqs, resp)
    srv.close()


def test_overflow_while_others_run_stays_within_budget(env):
    """Every class starts with a 65536-entry workspace and overflows on its first
    frame while other frames of the burst are in flight; each overflowed request
    is admitted again through the budget, so the peak never exceeds it."""
    rgs = env["rgs"]
    reqs = schedule(env, 12, rate=1000.0, burst=12, seed=11)
    budget = 1 << 30
    _log(f"[serve] overflow under load: 12 requests at once, budget {budget} bytes")
    srv = rgs.Server(0, n_streams=4, mem_budget=budget, use_graphs=True, entries_per_gaussian=0.01)
    resp, st = srv.serve(reqs)
    _log(f"[serve] {st}; retried {[r['retried'] for r in resp]}")
    assert sum(r["retried"] for r in resp) >= 2
    assert st["max_in_flight"] >= 2
    assert st["ws_bytes_peak"] <= budget
    assert_same_as_alone(env, reqs, resp)
    srv.close()


def test_budget_admits_one_workspace_at_a_time(env):
    rgs, torch = env["rgs"], env["torch"]
    from paper_2608_15785_amd import _binding as B
    epg = 12.0
    n0, n1 = env["scenes"][0].n, env["scenes"][1].n
    sizes = {
        (0, 1280, 720): B.workspace_size(n0, 1280, 720, "fast", max(65536, math.ceil(epg * n0))),
        (1, 1920, 1080): B.workspace_size(n1, 1920, 1080, "fast", max(65536, math.ceil(epg * n1))),
    }
    budget = int(max(sizes.values()) * 1.05)
    big = B.workspace_size(n1, 3840, 2160, "fast", max(65536, math.ceil(epg * n1)))
    assert big > budget
    reqs = []
    plan = [(0, 1280, 720), (1, 1920, 1080), (0, 1280, 720), (1, 3840, 2160), (1, 1920, 1080), (0, 1280, 720)]
    for k, (s, W, H) in enumerate(plan):
        cam = wl.serving_camera(s, 3 * k, W, H)
        out = torch.full((3, H, W), float("nan"), dtype=torch.float32, device="cuda:0")
        reqs.append((env["dev"][s], cam, "fast", 0.0, out))
    _log(f"[serve] budget {budget} bytes for classes {sizes}, 4K request needs {big}")
    srv = rgs.Server(0, n_streams=4, mem_budget=budget, use_graphs=True, entries_per_gaussian=epg)
    resp, st = srv.serve(reqs)
    _log(f"[serve] {st}")
    assert resp[3]["status"] == B.RGS_E_OOM
    assert st["ws_bytes_peak"] <= budget
    assert st["n_evicted"] >= 3
    assert st["max_in_flight"] == 1
    ok = [i for i in range(len(reqs)) if i != 3]
    assert_same_as_alone(env, [reqs[i] for i in ok], [resp[i] for i in ok])
    srv.close()


def test_small_request_in_the_mix_matches_the_oracle(env):
    rgs, torch = env["rgs"], env["torch"]
    reqs = schedule(env, 8, rate=3000.0, burst=8, seed=9)
    cam = wl.config_camera("small")
    out = torch.full((3, cam.height, cam.width), float("nan"), dtype=torch.float32, device="cuda:0")
    reqs.insert(3, (env["dsmall"], cam, "fast", 0.0, out))
    _log("[serve] 9 requests, one of them the 10k-Gaussian 256x256 frame")
    srv = rgs.Server(0, n_streams=4, mem_budget=24 << 30, use_graphs=True, entries_per_gaussian=12.0)
    resp, st = srv.serve(reqs)
    torch.cuda.synchronize()
    assert all(r["status"] == 0 for r in resp)
    fr = oracle_frame(env["small"], cam, "fast")
    rep = compare_image(out.cpu().numpy(), fr, "fast")
    _log(f"[serve] small request vs oracle: {rep}")
    assert_same_as_alone(env, reqs, resp)
    srv.close()


def test_malformed_schedules_are_rejected(env):
    rgs, torch = env["rgs"], env["torch"]
    from paper_2608_15785_amd import _binding as B
    ds = env["dev"][0]
    cam = wl.serving_camera(0, 0, 64, 48)
    out = torch.zeros((3, 48, 64), dtype=torch.float32, device="cuda:0")
    srv = rgs.Server(0, n_streams=2, mem_budget=1 << 30)
    with pytest.raises(rgs.RGSError) as e:
        srv.serve([(ds, cam, "fast", 0.5, out), (ds, cam, "fast", 0.1, out)])
    assert e.value.status == B.RGS_E_INVALID
    bad = wl.serving_camera(0, 0, 64, 48)
    bad.z_near = -1.0
    with pytest.raises(rgs.RGSError) as e:
        srv.serve([(ds, bad, "fast", 0.0, out)])
    assert e.value.status == B.RGS_E_INVALID
    resp, st = srv.serve([])
    assert resp == [] and st["n_captured"] == 0
    srv.close()
