"""Serving engine (include/ctserve.h) on the GPU: requests of mixed geometries, methods,
directions and storage types arrive in a burst while earlier calls are still running; queued
requests that share a plan are merged into batched calls, calls overlap on the slots' streams,
admission waits for arena memory; every result is bitwise the one the request gets alone
(direct ctp_project / ctp_backproject, batch 1), and served FP32 results meet the oracle bar."""
import math

import numpy as np
import pytest

from paper_2503_16741_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2503_16741_amd import ctproj
    ctproj.lib()
    return torch


def geometries():
    th = synth.full_circle(24)
    fan = synth.Geometry(kind="fan2d", det="flat", nx=40, ny=36, nz=1, dx=1.0, dy=1.0, dz=1.0,
                         nu=96, nv=1, du=1.2, dv=1.0, n_views=24, theta=th, sad=150.0, sdd=300.0,
                         u_ofst=0.3)
    cone = dict(kind="cone", nx=28, ny=26, nz=18, dx=0.9, dy=0.9, dz=1.0, nu=64, nv=40, du=1.0,
                dv=1.0, n_views=20, theta=synth.full_circle(20), sad=160.0, sdd=280.0)
    flat = synth.Geometry(det="flat", x_src=0.7, **cone)
    curved = synth.Geometry(det="curved", **cone)
    rng = np.random.default_rng(5)
    nc = dict(cone, kind="cone_noncirc")
    noncirc = synth.Geometry(det="flat", phi=rng.uniform(-0.03, 0.03, 20),
                             psi=rng.uniform(-0.03, 0.03, 20), z_src=rng.uniform(-2, 2, 20), **nc)
    big = synth.Geometry(kind="cone", det="flat", nx=128, ny=128, nz=128, dx=0.5, dy=0.5,
                         dz=0.5, nu=256, nv=200, du=0.5, dv=0.5, n_views=300,
                         theta=synth.full_circle(300), sad=300.0, sdd=500.0)
    return {"fan": (fan, "sf"), "fan_dd": (fan, "dd"), "flat": (flat, "sf"),
            "curved_dd": (curved, "dd"), "noncirc": (noncirc, "sf"), "big": (big, "sf"),
            "curved_recon": (curved, "sf", "recon")}


def make_plan(ctproj, entry):
    g, m = entry[0], entry[1]
    return ctproj.ctp_plan_create(g, m, entry[2] if len(entry) > 2 else "proj")


def alone(ctproj, plan, direction, x, out_dtype):
    return (ctproj.project(plan, x, out_dtype=out_dtype) if direction == "forward"
            else ctproj.backproject(plan, x, out_dtype=out_dtype))


def make_input(torch, geom, direction, dtype, seed):
    a = (synth.random_volume(geom, seed=seed) if direction == "forward"
         else synth.random_sinogram(geom, seed=seed))
    return torch.from_numpy(a).cuda().to(dtype).contiguous()


@pytest.mark.parametrize("n_slots,express,sliced", [(2, False, False), (3, True, False),
                                                    (4, True, True)])
def test_mixed_burst_alone_equals_in_mix(torch_gpu, orc, n_slots, express, sliced):
    """Every result of a mixed burst equals the direct batch-1 call bit for bit; with an
    express slot (the last one, for the small kinds only) the long calls never run there and
    run one at a time.  Sliced: every call is split into launches of a few views (the long
    ones into one launch per view), with the same bits."""
    torch = torch_gpu
    from paper_2503_16741_amd import ctproj
    geo = geometries()
    plans = {k: make_plan(ctproj, e) for k, e in geo.items()}
    work = {k: float(e[0].n_vox) * e[0].n_views for k, e in geo.items()}
    small_work = max(w for k, w in work.items() if k != "big")
    assert small_work < work["big"]
    srv = ctproj.Server(256 << 20, n_slots=n_slots, max_batch=6,
                        express_work=small_work if express else 0.0,
                        launch_work=small_work / 5 if sliced else 0.0)
    rng = np.random.default_rng(42)
    reqs = []
    # four long calls first (two run, two wait), so that the burst behind them queues and
    # gets merged
    for i in range(4):
        reqs.append(("big", "forward", torch.float32, torch.float32, 1000 + i))
    kinds = ["fan", "fan_dd", "flat", "curved_dd", "noncirc", "curved_recon"]
    for i in range(60):
        k = kinds[int(rng.integers(len(kinds)))]
        d = "forward" if rng.random() < 0.5 else "backward"
        u = rng.random()
        dt = torch.float32 if u < 0.5 else torch.bfloat16 if u < 0.8 else torch.float16
        odt = dt if rng.random() < 0.7 else torch.float32
        reqs.append((k, d, dt, odt, i))
    inputs = [make_input(torch, geo[k][0], d, dt, seed) for (k, d, dt, odt, seed) in reqs]
    torch.cuda.synchronize()
    print(f"serving burst: {len(reqs)} requests", flush=True)
    tickets = [srv.submit(plans[k], d, x, out_dtype=odt)
               for (k, d, dt, odt, seed), x in zip(reqs, inputs)]
    served, infos = [], []
    for t in tickets:
        served.append(srv.wait(t, timeout_s=60).clone())
        infos.append(srv.info(t))
    torch.cuda.synchronize()
    for t in tickets:
        srv.release(t)
    stats = srv.stats()
    print("server stats", stats, flush=True)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["max_batch_seen"] > 1, "no requests were merged"
    assert stats["max_running"] > 1, "no calls overlapped"
    assert any(i["batch"] > 1 for i in infos)
    for i in infos:
        assert i["submit_ns"] <= i["admit_ns"] <= i["done_ns"]
    if express:
        assert all(i["slot"] != n_slots - 1 for r, i in zip(reqs, infos) if r[0] == "big")
        assert any(i["slot"] == n_slots - 1 for i in infos)
        # one interval per call (merged requests share theirs)
        big = sorted({(i["admit_ns"], i["done_ns"]) for r, i in zip(reqs, infos) if r[0] == "big"})
        assert all(a[1] <= b[0] for a, b in zip(big, big[1:])), "long calls overlapped"
    # bitwise: alone (batch 1, direct call) == in the mix
    for (k, d, dt, odt, seed), x, y in zip(reqs, inputs, served):
        ref = alone(ctproj, plans[k], d, x, odt)
        torch.cuda.synchronize()
        assert y.dtype == ref.dtype and y.shape == ref.shape
        assert torch.equal(y, ref), (k, d, dt, odt, seed)
    # the FP32 bar against the oracle for one served request of each small kind
    seen = set()
    for (k, d, dt, odt, seed), x, y in zip(reqs, inputs, served):
        if k == "big" or dt != torch.float32 or odt != torch.float32 or (k, d) in seen:
            continue
        seen.add((k, d))
        g, m = geo[k][0], geo[k][1]
        mode = geo[k][2] if len(geo[k]) > 2 else "proj"
        xin = x.cpu().numpy()
        ref = (orc.forward(g, xin, method=m, mode=mode) if d == "forward"
               else orc.adjoint(g, xin, method=m, mode=mode))
        err = float(np.max(np.abs(y.cpu().numpy() - ref)) / max(np.max(np.abs(ref)), 1e-30))
        assert err <= TOL, (k, d, err)
    assert len(seen) >= 7
    srv.close()


def test_admission_waits_for_memory(torch_gpu):
    """An arena that holds about two requests: the rest wait in the queue and run as outputs are
    released; a request that can never fit is refused at submission."""
    torch = torch_gpu
    from paper_2503_16741_amd import ctproj
    g, m = geometries()["flat"][:2]
    plan = ctproj.ctp_plan_create(g, m)
    vb, sb = ctproj.ctp_plan_bytes(plan, 1)
    ws = ctproj.ctp_workspace_bytes(plan, ctproj.CTP_FORWARD, 1)
    per = (sb + 255) // 256 * 256 + (ws + 255) // 256 * 256
    arena = 2 * per + 4096
    srv = ctproj.Server(arena, n_slots=4, max_batch=4)
    xs = [make_input(torch, g, "forward", torch.float32, 70 + i) for i in range(8)]
    torch.cuda.synchronize()
    tickets = [srv.submit(plan, "forward", x) for x in xs]
    outs = []
    for t in tickets:          # each output is copied out and released before the next wait
        outs.append(srv.wait(t, timeout_s=60).clone())
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == 8 and st["arena_peak"] <= arena
    for x, y in zip(xs, outs):
        assert torch.equal(y, ctproj.project(plan, x))
    # a request whose output alone exceeds the arena
    big = ctproj.ctp_plan_create(geometries()["big"][0], "sf")
    xb = make_input(torch, big.geom, "forward", torch.float32, 99)
    with pytest.raises(ctproj.CtpError) as e:
        srv.submit(big, "forward", xb)
    assert e.value.status == ctproj.CTP_ENOMEM
    # a wait that times out leaves the request queued or running; a released ticket is gone
    t = srv.submit(plan, "forward", xs[0])
    try:
        y = srv.wait(t, timeout_s=0.0)
    except ctproj.CtpError as err:
        assert err.status == ctproj.CTP_ETIMEOUT
        y = srv.wait(t, timeout_s=60)
    assert torch.equal(y, outs[0])
    srv.release(t)
    with pytest.raises(ctproj.CtpError):
        srv.release(t)
    srv.close()


def test_results_stay_resident(torch_gpu):
    """Outputs keep their values while later requests run, until released."""
    torch = torch_gpu
    from paper_2503_16741_amd import ctproj
    g, m = geometries()["fan"][:2]
    plan = ctproj.ctp_plan_create(g, m)
    srv = ctproj.Server(64 << 20, n_slots=3, max_batch=8)
    x0 = make_input(torch, g, "forward", torch.float32, 3)
    t0 = srv.submit(plan, "forward", x0)
    y0 = srv.wait(t0, timeout_s=60)
    keep = y0.clone()
    later = [srv.submit(plan, "backward", make_input(torch, g, "backward", torch.float32, 10 + i))
             for i in range(20)]
    for t in later:
        srv.wait(t, timeout_s=60)
        srv.release(t)
    torch.cuda.synchronize()
    assert torch.equal(y0, keep)
    srv.release(t0)
    srv.close()
    assert math.isfinite(float(keep.abs().max()))
