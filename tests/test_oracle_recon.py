"""Pins of the oracle's FBP pieces ("recon" mode and the ramp filter), checked against what
the mathematics fixes rather than against the code's own formulas:

  R1  the sampled ramp kernels have the textbook frequency responses (Ram-Lak |f| up to the
      Nyquist frequency, Shepp-Logan |f| |sinc(f a)|);
  R2  "recon"-mode back projection of an all-ones sinogram equals sum_b (SAD / W_b)^2 at
      every voxel whose footprint lies on the detector (normalised interpolation weights),
      with W_b computed here from the scan geometry;
  R3  filtered back projection of exact (analytic, cell-averaged) projections of a uniform
      disc / ball reconstructs its density: fan beam flat and curved, both windows, and FDK
      on the central slice of a cone-beam scan, flat and curved;
  R4  the recon-mode forward projection is the exact transpose of its back projection.
A dropped factor (1/2, the magnification, the angular step, the cosine weight, the depth
weight) or a wrong sign moves R3 by far more than its tolerance.
"""
import math

import numpy as np
import pytest

from paper_2503_16741_amd import synth
import refs

from oracle.ramp import ramp_taps, ramp_filter


@pytest.mark.parametrize("window", ["ram-lak", "shepp-logan"])
def test_ramp_frequency_response(window):
    a, n = 0.7, 40001
    h = ramp_taps(n, a, window)
    k = np.arange(-(n - 1), n)
    for fa in (0.03, 0.1, 0.25, 0.37, 0.49):
        f = fa / a
        H = a * np.sum(h * np.cos(2 * np.pi * f * k * a))
        want = abs(f) if window == "ram-lak" else abs(f) * abs(np.sinc(f * a))
        assert abs(H - want) <= 1e-6 * abs(f) + 1e-7, (fa, H, want)


def fan(det, n_views=360):
    return synth.Geometry(kind="fan2d", det=det, nx=64, ny=64, nz=1, dx=1.0, dy=1.0, dz=1.0,
                          nu=200, nv=1, du=1.0, dv=1.0, n_views=n_views,
                          theta=synth.full_circle(n_views), sad=200.0, sdd=400.0)


def cone(det, n_views=180):
    return synth.Geometry(kind="cone", det=det, nx=32, ny=32, nz=12, dx=1.0, dy=1.0, dz=1.0,
                          nu=110, nv=32, du=1.0, dv=1.0, n_views=n_views,
                          theta=synth.full_circle(n_views), sad=200.0, sdd=400.0)


@pytest.mark.parametrize("det", ["flat", "curved"])
@pytest.mark.parametrize("kind", ["fan2d", "cone"])
def test_recon_weights_sum(orc, det, kind):
    g = synth.Geometry(kind=kind, det=det, nx=9, ny=8, nz=5, dx=1.1, dy=0.9, dz=1.2, nu=80,
                       nv=50, du=1.0, dv=1.0, n_views=11, theta=synth.full_circle(11) + 0.1,
                       sad=60.0, sdd=130.0, x_ofst=1.5, y_ofst=-1.0, z_ofst=0.5, u_ofst=0.4,
                       v_ofst=-0.3, z_src=0.8 if kind == "cone" else 0.0)
    ones = np.ones(g.sino_shape)
    got = orc.adjoint(g, ones, mode="recon")
    nz = g.nz if kind == "cone" else 1
    want = np.zeros((nz, g.ny, g.nx))
    for b in range(g.n_views):
        s, d, eu, ev, n = refs._frame(g, b)[:5]
        for iz in range(nz):
            for iy in range(g.ny):
                for ix in range(g.nx):
                    c = np.array([(ix - (g.nx - 1) / 2) * g.dx + 1.5,
                                  (iy - (g.ny - 1) / 2) * g.dy - 1.0,
                                  ((iz - (nz - 1) / 2) * g.dz + 0.5) if kind == "cone" else 0.0])
                    w = np.dot(s - c, n)
                    if det == "curved":
                        w = math.hypot(np.dot(c - s, eu), w)
                    want[iz, iy, ix] += (60.0 / w) ** 2
    assert np.max(np.abs(got.reshape(want.shape) - want)) <= 1e-12 * np.max(want)


def _disc_sino(g, centre, radius, half_height, sub_v):
    ells = [dict(rho=1.0, centre=np.asarray(centre, float),
                 axes=np.array([radius, radius, half_height]), rot=np.eye(3))]
    p = np.array(refs.ellipsoid_cell_average(g, ells, range(g.n_views), sub_u=8, sub_v=sub_v))
    return p.reshape(g.sino_shape)


@pytest.mark.parametrize("window", ["ram-lak", "shepp-logan"])
@pytest.mark.parametrize("det", ["flat", "curved"])
def test_fbp_uniform_disc(orc, det, window):
    g = fan(det)
    c, r = (3.0, -2.0, 0.0), 20.0
    x = orc.fbp(g, _disc_sino(g, c, r, 1e6, 1), window)
    X, Y = np.meshgrid((np.arange(64) - 31.5), (np.arange(64) - 31.5))
    rr = np.hypot(X - c[0], Y - c[1])
    assert np.max(np.abs(x[rr < r - 3] - 1.0)) <= 1e-3
    assert np.max(np.abs(x[rr > r + 3])) <= 2e-2


@pytest.mark.parametrize("det", ["flat", "curved"])
def test_fdk_uniform_ball_central_slice(orc, det):
    g = cone(det)
    c, r = (1.5, -1.0, 0.0), 10.0
    sino = _disc_sino(g, c, r, r, 2)
    mid = [g.nz // 2 - 1, g.nz // 2]
    X, Y = np.meshgrid((np.arange(32) - 15.5), (np.arange(32) - 15.5))
    rr = np.hypot(X - c[0], Y - c[1])
    inside = np.flatnonzero((rr < 5.0).ravel())
    for iz in mid:
        zc = (iz - (g.nz - 1) / 2)
        vox = iz * g.nx * g.ny + inside
        x = orc.fbp(g, sino, "ram-lak", voxels=vox)
        # density 1 inside the ball; the slice cuts it at |z| = 0.5 mm
        assert abs(zc) < 1.0
        assert np.max(np.abs(x - 1.0)) <= 5e-3, (iz, float(np.max(np.abs(x - 1.0))))


@pytest.mark.parametrize("kind", ["fan2d", "cone"])
def test_recon_mode_adjoint_identity(orc, kind):
    g = synth.Geometry(kind=kind, det="flat", nx=10, ny=9, nz=6, dx=1.0, dy=1.0, dz=1.0, nu=40,
                       nv=24, du=1.0, dv=1.0, n_views=5, theta=synth.full_circle(5) + 0.3,
                       sad=50.0, sdd=100.0, x_src=0.7, u_ofst=0.2)
    rng = np.random.default_rng(3)
    x = rng.random(g.vol_shape)
    y = rng.random(g.sino_shape)
    lhs = np.sum(orc.forward(g, x, mode="recon") * y)
    rhs = np.sum(x * orc.adjoint(g, y, mode="recon"))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_recon_mode_scope(orc):
    g = synth.noncirc_c4()
    g2 = fan("flat", 4)
    with pytest.raises(NotImplementedError):
        orc.adjoint(g2, np.zeros(g2.sino_shape), method="dd", mode="recon")
    with pytest.raises(NotImplementedError):
        ramp_filter(g, np.zeros((1,) + g.sino_shape[1:]))
