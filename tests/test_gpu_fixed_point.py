"""The forward projector's fixed-point accumulators at the edge of their range.

Every weight of the projector is non-negative, so for |x| <= X the largest possible sum in a
detector cell is X times the projection of the uniform unit volume: a volume that is X
everywhere reaches the true maximum of every cell, which the per-item scale 2^S (set from
max |x| and the plan's bound on the cell sum, Eq. 1 accumulated in 32-bit integers) must keep
below 2^31.  These cases project such uniform volumes -- SF and DD on the 256^3 x 360-view
and the curved 512x512x256 x 720-view scans at full size, and a recon-mode plan with strong
magnification and fine detector pitch, whose normalised weights sum to more per cell --
and compare sampled views with the FP64 oracle at the 1e-4 bar.
"""
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


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30))


def project(torch, plan, value, mode_note=""):
    from paper_2503_16741_amd import ctproj
    g = plan.geom
    v = torch.full(tuple(g.vol_shape), value, dtype=torch.float32, device="cuda")
    s = torch.full(tuple(g.sino_shape), float("nan"), dtype=torch.float32, device="cuda")
    ctproj.ctp_project(plan, v, s)
    torch.cuda.synchronize()
    return s.cpu().numpy()


@pytest.mark.parametrize("scan,method,views", [
    ("c2", "sf", [0, 45, 301]), ("c2", "dd", [0, 45, 301]),
    ("c3", "sf", [0, 333]), ("c3", "dd", [90, 500]),
])
def test_uniform_full_scale_volume(torch_gpu, orc, scan, method, views):
    from paper_2503_16741_amd import ctproj
    g = {"c2": synth.cone_c2, "c3": synth.curved_c3}[scan]()
    value = 3.0e4       # any value: the scale adapts to max |x|; all voxels sit at the maximum
    print(f"[fixed-point] uniform {scan} {method} x = {value}", flush=True)
    plan = ctproj.ctp_plan_create(g, method)
    y = project(torch_gpu, plan, value)
    assert np.all(np.isfinite(y))
    sel = np.asarray(views)
    ref = orc.forward(g, np.full(g.vol_shape, value, np.float32), method=method, views=sel)
    err = rel_err(y[sel], ref)
    print(f"[fixed-point] {scan} {method}: max cell {ref.max():.4g}, err {err:.2e}", flush=True)
    assert err <= TOL
    plan.close()


def test_uniform_volume_recon_mode_strong_magnification(torch_gpu, orc):
    """Recon mode normalises each footprint to unit sum and weights it by (SAD / W)^2: with
    magnification above 4 and detector cells of 0.28 mm under 0.5 mm voxels (footprints of
    about 12 columns) the cell sums are largest relative to the voxel count."""
    from paper_2503_16741_amd import ctproj
    n = 24
    g = synth.Geometry(kind="cone", det="flat", nx=n, ny=n, nz=n, dx=0.5, dy=0.5, dz=0.5,
                       nu=280, nv=200, du=0.28, dv=0.28, n_views=12,
                       theta=synth.full_circle(12) + 0.1, sad=100.0, sdd=400.0)
    plan = ctproj.ctp_plan_create(g, "sf", "recon")
    for value in (1.0, 2.5e30):
        y = project(torch_gpu, plan, value)
        ref = orc.forward(g, np.full(g.vol_shape, value, np.float32), mode="recon")
        err = rel_err(y, ref)
        print(f"[fixed-point] recon x = {value}: max cell {ref.max():.4g}, err {err:.2e}",
              flush=True)
        assert err <= TOL
    plan.close()


def test_uniform_volume_2d_coarse_and_fine_detector(torch_gpu, orc):
    """2D fan: the cell sum is a cell average of the footprints, so it stays near the path
    length whether detector cells are much coarser or finer than the pixels' shadows."""
    from paper_2503_16741_amd import ctproj
    for du in (3.0, 0.3):
        nu = int(math.ceil(300.0 / du))
        g = synth.Geometry(kind="fan2d", det="flat", nx=96, ny=96, nz=1, dx=1.0, dy=1.0, dz=1.0,
                           nu=nu, nv=1, du=du, dv=1.0, n_views=20,
                           theta=synth.full_circle(20), sad=500.0, sdd=1000.0)
        for method in ("sf", "dd"):
            plan = ctproj.ctp_plan_create(g, method)
            y = project(torch_gpu, plan, 1.0)
            ref = orc.forward(g, np.ones(g.vol_shape, np.float32), method=method)
            err = rel_err(y, ref)
            print(f"[fixed-point] 2D du {du} {method}: max cell {ref.max():.4g}, err {err:.2e}",
                  flush=True)
            assert err <= TOL
            plan.close()
