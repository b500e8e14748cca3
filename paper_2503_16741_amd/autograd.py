"""Differentiable projector on top of the C ABI (paper, Section 2.1 and Eq. 2).

``Projector(geom, 'proj', 'SF'|'DD', 'forward'|'backward')`` mirrors the paper's projector
module: a ``torch.nn.Module`` whose forward calls the library's projector and whose
autograd backward calls the matched adjoint (the gradient of y = A x with respect to x is
A^T, and that of x = A^T y with respect to y is A, Section 2.3).  Inputs are batched and
channelled tensors ``[B, C, *vol_shape]`` (or ``[B, C, *sino_shape]``), flattened to B*C items
for the library, as in the paper's Section 2.4 example.

``wls_loss`` is the weighted least-squares data term 0.5 * sum w (A x - y)^2 used for
model-based iterative reconstruction; its gradient A^T (w (A x - y)) comes out of autograd.
"""
from __future__ import annotations

import torch

from . import ctproj
from .synth import Geometry


def _flat(t: torch.Tensor, inner: tuple) -> tuple:
    lead = tuple(t.shape[:t.dim() - len(inner)])
    if tuple(t.shape[t.dim() - len(inner):]) != tuple(inner):
        raise ValueError(f"expected [...]+{tuple(inner)}, got {tuple(t.shape)}")
    return lead, t.reshape((-1,) + tuple(inner))


def _project(plan, x):
    g = plan.geom
    lead, xf = _flat(x.contiguous(), g.vol_shape)
    y = torch.empty((xf.shape[0],) + tuple(g.sino_shape), dtype=torch.float32, device=x.device)
    ctproj.ctp_project(plan, xf, y)
    return y.reshape(lead + tuple(g.sino_shape))


def _backproject(plan, y):
    g = plan.geom
    lead, yf = _flat(y.contiguous(), g.sino_shape)
    x = torch.empty((yf.shape[0],) + tuple(g.vol_shape), dtype=torch.float32, device=y.device)
    ctproj.ctp_backproject(plan, yf, x)
    return x.reshape(lead + tuple(g.vol_shape))


class ProjectFn(torch.autograd.Function):
    """y = A x; backward: grad_x = A^T grad_y."""

    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return _project(plan, x)

    @staticmethod
    def backward(ctx, gy):
        return _backproject(ctx.plan, gy), None


class BackprojectFn(torch.autograd.Function):
    """x = A^T y; backward: grad_y = A grad_x."""

    @staticmethod
    def forward(ctx, y, plan):
        ctx.plan = plan
        return _backproject(plan, y)

    @staticmethod
    def backward(ctx, gx):
        return _project(ctx.plan, gx), None


class Projector(torch.nn.Module):
    """Projector(geom, mode, method, direction) with mode 'proj' (standard projection) or
    'recon' (the depth-weighted back projection of FBP and its transpose; SF on circular
    scans), method 'SF' or 'DD', direction 'forward' (A) or 'backward' (A^T)."""

    def __init__(self, geom: Geometry, mode: str = "proj", method: str = "SF",
                 direction: str = "forward"):
        super().__init__()
        if mode not in ("proj", "recon"):
            raise ValueError("mode must be 'proj' or 'recon'")
        if method.upper() not in ("SF", "DD"):
            raise NotImplementedError(f"projector method {method!r} is not built (SF, DD are)")
        if direction not in ("forward", "backward"):
            raise ValueError("direction must be 'forward' or 'backward'")
        self.geom = geom
        self.mode = mode
        self.method = method.lower()
        self.direction = direction
        self._plan = None

    @property
    def plan(self):
        if self._plan is None:
            self._plan = ctproj.ctp_plan_create(self.geom, self.method, self.mode)
        return self._plan

    def forward(self, t: torch.Tensor) -> torch.Tensor:
        if t.dtype != torch.float32:
            raise TypeError("the projector computes in float32")
        if self.direction == "forward":
            return ProjectFn.apply(t, self.plan)
        return BackprojectFn.apply(t, self.plan)


def wls_loss(A: Projector, x: torch.Tensor, y_hat: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """0.5 * sum w (A x - y_hat)^2 (weighted least squares data term)."""
    r = A(x) - y_hat
    return 0.5 * torch.sum(w * r * r)


def poisson_sinogram(line_integrals: torch.Tensor, i0: float, generator=None):
    """Transmission counts n ~ Poisson(I0 exp(-l)), the log estimate y_hat = -ln(max(n,1)/I0)
    and the WLS weights w = n."""
    counts = torch.poisson(i0 * torch.exp(-line_integrals), generator=generator)
    y_hat = -torch.log(torch.clamp(counts, min=1.0) / i0)
    return y_hat, counts
