"""Differentiable projector (paper, Sections 2.1 and 2.4; Eq. 2): the autograd backward is the
hand-written adjoint kernel.  Checked by the dot-product test through autograd, by central
finite differences of the WLS loss (exact for a quadratic loss up to rounding) and against
the FP64 oracle's A^T (w (A x - y))."""
import numpy as np
import pytest

from paper_2503_16741_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def small(det="flat", kind="cone"):
    th = synth.full_circle(9) + 0.1
    if kind == "fan2d":
        return synth.Geometry(kind="fan2d", det=det, nx=20, ny=18, nz=1, dx=1.0, dy=1.0, dz=1.0,
                              nu=40, nv=1, du=1.2, dv=1.0, n_views=9, theta=th, sad=200.0,
                              sdd=400.0)
    return synth.Geometry(kind=kind, det=det, nx=14, ny=12, nz=10, dx=1.0, dy=1.0, dz=1.0,
                          nu=32, nv=24, du=1.1, dv=1.1, n_views=9, theta=th, sad=150.0,
                          sdd=280.0)


@pytest.mark.parametrize("method", ["SF", "DD"])
@pytest.mark.parametrize("kind,det", [("cone", "flat"), ("cone", "curved"), ("fan2d", "flat")])
def test_autograd_dot_product(torch_gpu, method, kind, det):
    """<A x, y> = <x, A^T y> where A^T y comes from autograd of <A x, y>."""
    torch = torch_gpu
    from paper_2503_16741_amd.autograd import Projector
    g = small(det, kind)
    A = Projector(g, "proj", method, "forward")
    gen = torch.Generator(device="cuda").manual_seed(0)
    x = torch.rand((2, 3) + g.vol_shape, device="cuda", generator=gen).requires_grad_(True)
    y = torch.rand((2, 3) + g.sino_shape, device="cuda", generator=gen)
    lhs = torch.sum(A(x).double() * y.double())
    (gx,) = torch.autograd.grad(torch.sum(A(x) * y), [x])
    rhs = torch.sum(x.detach().double() * gx.double())
    assert abs(float(lhs - rhs)) <= 1e-5 * abs(float(lhs))
    At = Projector(g, "proj", method, "backward")
    yv = y.clone().requires_grad_(True)
    (gy,) = torch.autograd.grad(torch.sum(At(yv) * x.detach()), [yv])
    assert abs(float(torch.sum(gy.double() * y.double()) - lhs)) <= 1e-5 * abs(float(lhs))


def test_wls_gradient_matches_oracle_and_fd(torch_gpu, orc):
    """The WLS gradient A^T (w (A x - y)) through autograd against the FP64 oracle, and against
    a central difference of the loss.
    - gradient: the tolerance follows from the parity bar eps = 1e-4 (max error / max value of
      each FP32 projection): eps for the back projection plus eps max|A x| carried through
      A^T w, i.e. eps (1 + max A^T (w max|A x|) / max|g|);
    - central difference: the loss is quadratic, so the difference quotient is exact up to the
      errors of the two FP32 losses and of the FP32 gradient.  Each loss errs by
      sum w (r delta + delta^2 / 2) (delta: the FP32 projection's error in each cell, measured
      against the oracle on the same inputs, r: the residual) plus its FP32 summation (1e-6 L);
      the analytic side by sum |g - g_oracle| |d|.  The bound is the sum of these."""
    torch = torch_gpu
    from paper_2503_16741_amd.autograd import Projector, wls_loss, poisson_sinogram
    eps = 1e-4
    g = small("curved")
    A = Projector(g, "proj", "SF", "forward")
    x_true = torch.from_numpy(0.02 * synth.phantom(g, seed=3)).cuda()
    gen = torch.Generator(device="cuda").manual_seed(1)
    y_hat, counts = poisson_sinogram(A(x_true), 1e5, generator=gen)
    x = torch.from_numpy(0.01 * synth.random_volume(g, seed=4)).cuda().requires_grad_(True)
    loss = wls_loss(A, x, y_hat, counts)
    (gx,) = torch.autograd.grad(loss, [x])
    # oracle: A^T (w (A x - y)) in FP64 on the same inputs
    xn = x.detach().cpu().numpy().astype(np.float64)
    yh, w = y_hat.cpu().numpy().astype(np.float64), counts.cpu().numpy().astype(np.float64)
    ax = orc.forward(g, xn)
    ref = orc.adjoint(g, w * (ax - yh))
    gmax = np.max(np.abs(ref))
    tol_g = eps * (1.0 + np.max(orc.adjoint(g, w * np.max(np.abs(ax)))) / gmax)
    gn = gx.cpu().numpy().astype(np.float64)
    err = np.max(np.abs(gn - ref)) / gmax
    print(f"[autograd] gradient err {err:.2e} (bound {tol_g:.2e})", flush=True)
    assert err <= tol_g
    # central difference along a random direction
    dn = (synth.random_volume(g, seed=5) - 0.5).astype(np.float32)
    d = torch.from_numpy(dn).cuda()
    h = 1e-2
    bound = float(np.sum(np.abs(gn - ref) * np.abs(dn)))
    losses = []
    for sgn in (1.0, -1.0):
        xs = x.detach() + sgn * h * d
        with torch.no_grad():
            losses.append(float(wls_loss(A, xs, y_hat, counts).double()))
            a_gpu = A(xs).cpu().numpy().astype(np.float64)
        a = orc.forward(g, xs.cpu().numpy().astype(np.float64))
        r, delta = a - yh, a_gpu - a
        lval = 0.5 * np.sum(w * r * r)
        bound += (np.sum(w * np.abs(r * delta + 0.5 * delta * delta)) + 1e-6 * lval) / (2 * h)
    fd = (losses[0] - losses[1]) / (2 * h)
    an = float(torch.sum(gx.double() * d.double()))
    print(f"[autograd] fd {fd:.6e} analytic {an:.6e}: |diff| {abs(fd - an):.3e} "
          f"(bound {bound:.3e}, {bound / abs(an):.2e} relative)", flush=True)
    assert abs(fd - an) <= bound


def test_mbir_descent(torch_gpu):
    """A few gradient steps of WLS reconstruction lower the loss (Section 2.4 example)."""
    torch = torch_gpu
    from paper_2503_16741_amd.autograd import Projector, wls_loss, poisson_sinogram
    g = small()
    A = Projector(g, "proj", "SF", "forward")
    x_true = torch.from_numpy(0.02 * synth.phantom(g, seed=6)).cuda()
    gen = torch.Generator(device="cuda").manual_seed(2)
    y_hat, w = poisson_sinogram(A(x_true), 1e5, generator=gen)
    x = torch.zeros_like(x_true, requires_grad=True)
    opt = torch.optim.Adam([x], lr=2e-3)
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss = wls_loss(A, x, y_hat, w)
        loss.backward()
        opt.step()
        losses.append(loss.item())
    assert losses[-1] < 0.2 * losses[0]
