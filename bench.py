#!/usr/bin/env python3
"""Benchmark: FP32 separable-footprint (SF-TT) forward + back projection on one MI355X.

Workload (one "step"): SF forward projection followed by SF back projection of a seeded
synthetic ellipsoid phantom, 256^3 voxels at 0.5 mm, 360 views over 360 deg, flat detector
512 x 384 at 0.8 mm, SAD 785 mm, SDD 1200 mm, inputs resident in HBM.  The metric is
voxel x view updates per second over the pair, GUPS = 2 * N_vox * N_view / t_pair, with p50/p99
pair latency.  Prints one JSON line.

The dominant kernel's roofline uses an algorithmic FP32 operation count per voxel-view of the
SF-TT method (constants below, measured footprint statistics from the CPU oracle) against the
chip's FP32 VALU issue rate; the CPU baseline times the FP64 oracle on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GUPS (voxel×view updates/s) SF fwd+back at 256³×360 views; p99 latency"

# Algorithmic FP32 operations per voxel-view of SF-TT on a circular scan (one direction):
#   axial corners 4 + corner sort 6 + trapezoid set-up 10 + 13 per interior row edge
#   + 1 per touched row + 2 per non-zero of A (weight product and multiply-add),
# with the footprint statistics of this scan measured by the oracle over 18 views:
#   touched rows per voxel-view 2.007, non-zeros per voxel-view 4.461
# (transaxial work is per voxel column and view, amortised over 256 slices: ~0.4).
SF_ROWS_PER_VV = 2.007
SF_NNZ_PER_VV = 4.461
SF_OPS_PER_VV = 4 + 6 + 10 + 13 * (SF_ROWS_PER_VV - 1) + SF_ROWS_PER_VV + 2 * SF_NNZ_PER_VV + 0.4
# FP32 VALU issue peak: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 lane-ops/s (one op per
# lane per clock; packed-FP32 dual issue is not used).
VALU_PEAK = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12

WORKLOAD = ("3D circular cone-beam SF-TT forward+back: 256^3 FP32 at 0.5 mm (20 seeded "
            "ellipsoids), 360 views/360 deg, flat 512x384 at 0.8 mm, SAD 785 mm, SDD 1200 mm")


def kernel_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "plan.cpp", "engine.h"):
        with open(os.path.join(ROOT, "paper_2503_16741_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name):
    """HBM bytes per launch from the committed PMC summary, if it was taken on this source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_hash():
        return None
    k = t.get("kernels", {}).get(kernel_name)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(geom, vol, n_views=32, n_vox=200000):
    """Time the FP64 oracle on a bounded sample of the same scan."""
    import numpy as np
    import oracle
    from paper_2503_16741_amd import synth
    views = np.linspace(0, geom.n_views - 1, n_views).astype(np.int32)
    t0 = time.perf_counter()
    oracle.forward(geom, vol, views=views)
    t1 = time.perf_counter()
    rng = np.random.default_rng(0)
    idx = rng.choice(geom.n_vox, size=n_vox, replace=False)
    ys = synth.random_sinogram(geom, seed=1)
    t2 = time.perf_counter()
    oracle.adjoint(geom, ys, voxels=idx)
    t3 = time.perf_counter()
    updates = n_views * geom.n_vox + n_vox * geom.n_views
    secs = (t1 - t0) + (t3 - t2)
    return {"value": updates / secs / 1e9, "unit": "GUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle: SF forward of the full 256^3 phantom for {n_views} of 360 "
                      f"views + SF adjoint at {n_vox} random voxels over all 360 views "
                      f"({updates:.3e} voxel-view updates in {secs:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dd", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(views would shard with no exchange; the adjoint needs one all-reduce)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2503_16741_amd import ctproj, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    g = synth.cone_c2()
    print(f"[bench] building phantom {g.nx}x{g.ny}x{g.nz}", file=sys.stderr, flush=True)
    vol_np = synth.phantom(g, seed=0)
    vol = torch.from_numpy(vol_np).to(dev)
    sino = torch.empty(g.sino_shape, dtype=torch.float32, device=dev)
    back = torch.empty(g.vol_shape, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def run(plan, steps, warmup, tag):
        for _ in range(warmup):
            ctproj.ctp_project(plan, vol, sino)
            ctproj.ctp_backproject(plan, sino, back)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            ctproj.ctp_project(plan, vol, sino)
            ev[k][1].record(stream)
            ctproj.ctp_backproject(plan, sino, back)
            ev[k][2].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fwd = np.array([e[0].elapsed_time(e[1]) for e in ev])
        bwd = np.array([e[1].elapsed_time(e[2]) for e in ev])
        pair = fwd + bwd
        print(f"[bench] {tag}: fwd {fwd.mean():.3f} ms, back {bwd.mean():.3f} ms, "
              f"wall {wall * 1e3 / steps:.3f} ms/step", file=sys.stderr, flush=True)
        return wall, fwd, bwd, pair

    plan = ctproj.ctp_plan_create(g, "sf")
    wall, fwd, bwd, pair = run(plan, args.steps, args.warmup, "SF")
    vv = float(g.n_vox) * g.n_views
    value = 2.0 * vv * args.steps / wall / 1e9
    dom_name, dom_ms = ("sf_forward", fwd.mean()) if fwd.mean() >= bwd.mean() else ("sf_backward", bwd.mean())
    ops = SF_OPS_PER_VV * vv
    achieved = ops / (dom_ms * 1e-3)
    traffic = load_traffic(dom_name)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "method": "sf", "batch": 1,
                   "vol": [g.nz, g.ny, g.nx], "views": g.n_views, "detector": [g.nv, g.nu]},
        "p50_ms": round(float(np.percentile(pair, 50)), 4),
        "p99_ms": round(float(np.percentile(pair, 99)), 4),
        "fwd_ms": round(float(fwd.mean()), 4),
        "back_ms": round(float(bwd.mean()), 4),
        "roofline": {
            "bound": "alu",
            "kernel": dom_name,
            "achieved": round(achieved / 1e12, 3),
            "peak": round(VALU_PEAK / 1e12, 2),
            "unit": "TFLOP/s",
            "frac": round(achieved / VALU_PEAK, 4),
            "ops_per_voxel_view": round(SF_OPS_PER_VV, 2),
            "traffic": traffic,
            "hbm_frac_algorithmic": round((vol.numel() + sino.numel()) * 4 / (dom_ms * 1e-3) / HBM_PEAK, 5),
        },
    }
    plan.close()

    if not args.no_dd:
        plan_dd = ctproj.ctp_plan_create(g, "dd")
        dsteps = max(3, args.steps // 4)
        wall_d, fwd_d, bwd_d, pair_d = run(plan_dd, dsteps, 1, "DD")
        out["dd"] = {"value": round(2.0 * vv * dsteps / wall_d / 1e9, 3), "unit": "GUPS",
                     "fwd_ms": round(float(fwd_d.mean()), 4),
                     "back_ms": round(float(bwd_d.mean()), 4),
                     "p99_ms": round(float(np.percentile(pair_d, 99)), 4)}
        plan_dd.close()

    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, vol_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
