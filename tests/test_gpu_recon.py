"""Recon mode and the ramp filter on the GPU against the FP64 oracle (bar: 1e-4 of the
maximum, FP32): the depth-weighted back projection of FBP and its transpose, the cosine-weighted
ramp filter, and filtered back projection end to end (fan beam and FDK, flat and curved)."""
import numpy as np
import pytest

from paper_2503_16741_amd import synth
import refs
from test_gpu_parity import small_geom, rel_err, run_fwd, run_bwd

pytestmark = pytest.mark.gpu
TOL = 1e-4
CIRC = [("fan2d", "flat"), ("fan2d", "curved"), ("cone", "flat"), ("cone", "curved")]


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2503_16741_amd import ctproj
    ctproj.lib()
    return torch


@pytest.mark.parametrize("kind,det", CIRC)
def test_recon_mode_parity(torch_gpu, orc, kind, det):
    from paper_2503_16741_amd import ctproj
    g = small_geom(kind, det, seed=31)
    plan = ctproj.ctp_plan_create(g, "sf", "recon")
    x = synth.random_volume(g, seed=32)
    y = synth.random_sinogram(g, seed=33)
    assert rel_err(run_fwd(torch_gpu, plan, x), orc.forward(g, x, mode="recon")) <= TOL
    assert rel_err(run_bwd(torch_gpu, plan, y), orc.adjoint(g, y, mode="recon")) <= TOL
    lhs = np.sum(run_fwd(torch_gpu, plan, x).astype(np.float64) * y)
    rhs = np.sum(x.astype(np.float64) * run_bwd(torch_gpu, plan, y))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("window", ["ram-lak", "shepp-logan"])
@pytest.mark.parametrize("kind,det", CIRC)
def test_ramp_filter_parity(torch_gpu, kind, det, window):
    torch = torch_gpu
    from paper_2503_16741_amd import ctproj
    from oracle.ramp import ramp_filter
    g = small_geom(kind, det, seed=34)
    plan = ctproj.ctp_plan_create(g, "sf")
    p = synth.random_sinogram(g, seed=35, batch=2)
    ref = ramp_filter(g, p, window)
    s = torch.from_numpy(p).cuda()
    out = torch.empty_like(s)
    ctproj.ctp_ramp_filter(plan, s, out, window)
    torch.cuda.synchronize()
    assert rel_err(out.cpu().numpy(), ref) <= TOL
    ctproj.ctp_ramp_filter(plan, s, s, window)            # in place
    torch.cuda.synchronize()
    assert torch.equal(s, out)
    # half-precision input, FP32 output: the filter of the rounded input
    sb = torch.from_numpy(p).cuda().to(torch.bfloat16)
    ctproj.ctp_ramp_filter(plan, sb, out, window)
    torch.cuda.synchronize()
    assert rel_err(out.cpu().numpy(), ramp_filter(g, sb.float().cpu().numpy(), window)) <= TOL


def _disc(g, c, r, hz, sub_v):
    ells = [dict(rho=1.0, centre=np.asarray(c, float), axes=np.array([r, r, hz]), rot=np.eye(3))]
    return np.array(refs.ellipsoid_cell_average(g, ells, range(g.n_views), sub_u=8,
                                                sub_v=sub_v)).reshape(g.sino_shape)


@pytest.mark.parametrize("det", ["flat", "curved"])
def test_fbp_fan_disc(torch_gpu, orc, det):
    torch = torch_gpu
    from paper_2503_16741_amd import ctproj
    g = synth.Geometry(kind="fan2d", det=det, nx=64, ny=64, nz=1, dx=1.0, dy=1.0, dz=1.0,
                       nu=200, nv=1, du=1.0, dv=1.0, n_views=360, theta=synth.full_circle(360),
                       sad=200.0, sdd=400.0)
    c, r = (3.0, -2.0, 0.0), 20.0
    p = _disc(g, c, r, 1e6, 1)
    plan = ctproj.ctp_plan_create(g, "sf", "recon")
    x = ctproj.fbp(plan, torch.from_numpy(p.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    ref = orc.fbp(g, p.astype(np.float32))
    assert rel_err(x, ref) <= TOL
    X, Y = np.meshgrid(np.arange(64) - 31.5, np.arange(64) - 31.5)
    assert np.max(np.abs(x[np.hypot(X - c[0], Y - c[1]) < r - 3] - 1.0)) <= 1e-3


@pytest.mark.parametrize("det", ["flat", "curved"])
def test_fdk_ball(torch_gpu, orc, det):
    torch = torch_gpu
    from paper_2503_16741_amd import ctproj
    g = synth.Geometry(kind="cone", det=det, nx=32, ny=32, nz=12, dx=1.0, dy=1.0, dz=1.0,
                       nu=110, nv=32, du=1.0, dv=1.0, n_views=180, theta=synth.full_circle(180),
                       sad=200.0, sdd=400.0)
    c, r = (1.5, -1.0, 0.0), 10.0
    p = _disc(g, c, r, r, 2).astype(np.float32)
    plan = ctproj.ctp_plan_create(g, "sf", "recon")
    x = ctproj.fbp(plan, torch.from_numpy(p).cuda())
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    assert rel_err(x, orc.fbp(g, p)) <= TOL
    X, Y = np.meshgrid(np.arange(32) - 15.5, np.arange(32) - 15.5)
    inside = np.hypot(X - c[0], Y - c[1]) < 5.0
    for iz in (g.nz // 2 - 1, g.nz // 2):
        assert np.max(np.abs(x[iz][inside] - 1.0)) <= 5e-3


def test_recon_projector_autograd(torch_gpu):
    """Projector(geom, 'recon', 'SF', 'backward') is differentiable; its gradient is the
    recon-mode forward projection (dot test through autograd)."""
    torch = torch_gpu
    from paper_2503_16741_amd.autograd import Projector
    g = small_geom("cone", "curved", seed=36)
    B = Projector(g, "recon", "SF", "backward")
    y = torch.from_numpy(synth.random_sinogram(g, seed=37, batch=2)).cuda().requires_grad_(True)
    w = torch.from_numpy(synth.random_volume(g, seed=38, batch=2)).cuda()
    loss = torch.sum(B(y) * w)
    loss.backward()
    lhs = float(torch.sum(y.grad.double() * y.detach().double()))
    assert abs(lhs - float(loss.detach())) <= 1e-5 * abs(lhs)
