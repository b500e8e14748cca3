"""Seeded synthetic inputs shared by the engine's tests, the benchmark and the oracle's tests.

This module holds scan *parameters* and *phantoms* only.  It contains none of the
projector arithmetic: no source/detector frames, no footprints, no weights.  Both the
HIP engine and the FP64 CPU oracle receive what is built here and expand it themselves.

Geometry parameters follow the paper's parameter table (Section 2.2, Table 1):
gantry angle theta, off-plane phi and in-plane psi rotations, SAD, SDD, source offsets
(x_src, z_src), object offsets (x_ofst, y_ofst, z_ofst) and detector offsets
(u_ofst, v_ofst).  Each per-view parameter is either a scalar (shared by every view) or a
vector with one entry per view (Section 2.2).

Phantoms are additive ellipses / ellipsoids with densities drawn from U[0, 1] and a
partial-volume voxelisation.  They stand in for the paper's bench-top CBCT, AAPM MAR and
XCAT data, none of which is available.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Union

import numpy as np

Param = Union[float, np.ndarray]

KINDS = ("fan2d", "cone", "cone_noncirc")
DETS = ("flat", "curved")
PER_VIEW = ("theta", "phi", "psi", "sad", "sdd", "x_src", "z_src",
            "x_ofst", "y_ofst", "z_ofst", "u_ofst", "v_ofst")


@dataclasses.dataclass
class Geometry:
    """Scan description: volume grid, detector grid and per-view parameters.

    Volume layout is ``[nz][ny][nx]`` (x fastest); sinogram layout is
    ``[n_views][nv][nu]`` (u fastest).  For ``fan2d`` nz = nv = 1.
    Lengths are in mm, angles in radians.
    """
    kind: str
    det: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    nu: int
    nv: int
    du: float
    dv: float
    n_views: int
    theta: Param = 0.0
    phi: Param = 0.0
    psi: Param = 0.0
    sad: Param = 500.0
    sdd: Param = 1000.0
    x_src: Param = 0.0
    z_src: Param = 0.0
    x_ofst: Param = 0.0
    y_ofst: Param = 0.0
    z_ofst: Param = 0.0
    u_ofst: Param = 0.0
    v_ofst: Param = 0.0

    def __post_init__(self):
        if self.kind not in KINDS:
            raise ValueError(f"kind must be one of {KINDS}, got {self.kind!r}")
        if self.det not in DETS:
            raise ValueError(f"det must be one of {DETS}, got {self.det!r}")
        for name in PER_VIEW:
            v = getattr(self, name)
            if isinstance(v, (list, tuple, np.ndarray)):
                arr = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
                setattr(self, name, arr)
            else:
                setattr(self, name, float(v))

    # -- plain data helpers (no projector arithmetic) --------------------------------
    def param(self, name: str) -> np.ndarray:
        """The parameter as a 1-D float64 array of length 1 (scalar) or n_views (vector)."""
        v = getattr(self, name)
        if isinstance(v, np.ndarray):
            return v
        return np.array([v], dtype=np.float64)

    def per_view(self, name: str) -> np.ndarray:
        """The parameter broadcast to one value per view."""
        v = self.param(name)
        if v.size == 1:
            return np.full(self.n_views, v[0], dtype=np.float64)
        if v.size != self.n_views:
            raise ValueError(f"{name} has {v.size} entries, expected 1 or {self.n_views}")
        return v

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx) if self.kind != "fan2d" else (self.ny, self.nx)

    @property
    def sino_shape(self):
        return ((self.n_views, self.nv, self.nu) if self.kind != "fan2d"
                else (self.n_views, self.nu))

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * (self.nz if self.kind != "fan2d" else 1)

    def subset_views(self, views) -> "Geometry":
        """The same scan restricted to the given view indices (an ordered subset)."""
        views = np.asarray(views, dtype=np.int64)
        kw = dataclasses.asdict(self)
        for name in PER_VIEW:
            v = getattr(self, name)
            if isinstance(v, np.ndarray) and v.size == self.n_views:
                kw[name] = v[views].copy()
        kw["n_views"] = int(views.size)
        return Geometry(**kw)


def full_circle(n_views: int) -> np.ndarray:
    """theta_k = 2*pi*k / n_views, k = 0..n_views-1."""
    return 2.0 * math.pi * np.arange(n_views, dtype=np.float64) / n_views


# -- the benchmark scans ---------------------------------------------------------------

def fan2d_c1() -> Geometry:
    """2D fan beam: 128x128 image at 1 mm, 180 views over 360 deg, flat 256 x 1 mm,
    SAD 500 mm, SDD 1000 mm."""
    return Geometry(kind="fan2d", det="flat", nx=128, ny=128, nz=1, dx=1.0, dy=1.0, dz=1.0,
                    nu=256, nv=1, du=1.0, dv=1.0, n_views=180, theta=full_circle(180),
                    sad=500.0, sdd=1000.0)


def cone_c2() -> Geometry:
    """3D circular cone beam: 256^3 at 0.5 mm, 360 views over 360 deg, flat detector
    512 columns x 384 rows at 0.8 mm, SAD 785 mm, SDD 1200 mm."""
    return Geometry(kind="cone", det="flat", nx=256, ny=256, nz=256, dx=0.5, dy=0.5, dz=0.5,
                    nu=512, nv=384, du=0.8, dv=0.8, n_views=360, theta=full_circle(360),
                    sad=785.0, sdd=1200.0)


def curved_c3() -> Geometry:
    """3D circular cone beam, curved detector 736 x 64 at 1.0 x 1.0 mm, 512x512x256 at
    0.5 mm, 720 views, SAD 595 mm, SDD 1085 mm."""
    return Geometry(kind="cone", det="curved", nx=512, ny=512, nz=256, dx=0.5, dy=0.5, dz=0.5,
                    nu=736, nv=64, du=1.0, dv=1.0, n_views=720, theta=full_circle(720),
                    sad=595.0, sdd=1085.0)


def serving_ladder() -> list:
    """Geometries a serving stream draws from: a 2D fan beam 256^2 at 0.5 mm with 360 views on
    a flat 512 x 1 mm detector (SAD 500, SDD 1000), and 3D circular cone beams 128^3, 256^3 and
    384^3 at 0.4 mm with 400 views on a flat 640 x 480 detector at 0.6 mm (SAD 785, SDD 1200)."""
    out = [("fan2d_256", Geometry(kind="fan2d", det="flat", nx=256, ny=256, nz=1, dx=0.5,
                                  dy=0.5, dz=1.0, nu=512, nv=1, du=1.0, dv=1.0, n_views=360,
                                  theta=full_circle(360), sad=500.0, sdd=1000.0))]
    for n in (128, 256, 384):
        out.append((f"cone_{n}", Geometry(kind="cone", det="flat", nx=n, ny=n, nz=n, dx=0.4,
                                          dy=0.4, dz=0.4, nu=640, nv=480, du=0.6, dv=0.6,
                                          n_views=400, theta=full_circle(400), sad=785.0,
                                          sdd=1200.0)))
    return out


def noncirc_c4(seed: int = 0) -> Geometry:
    """3D non-circular cone beam: 384^3 at 0.4 mm, 500 views, flat 640 x 480 at 0.6 mm,
    SAD 785 mm, SDD 1200 mm, with per-view seeded pose jitter: source offsets
    x_src, z_src ~ U[-5, 5] mm and detector tilts phi, psi ~ U[-2, 2] deg."""
    n = 500
    rng = np.random.default_rng(seed)
    x_src = rng.uniform(-5.0, 5.0, n)
    z_src = rng.uniform(-5.0, 5.0, n)
    phi = np.deg2rad(rng.uniform(-2.0, 2.0, n))
    psi = np.deg2rad(rng.uniform(-2.0, 2.0, n))
    return Geometry(kind="cone_noncirc", det="flat", nx=384, ny=384, nz=384,
                    dx=0.4, dy=0.4, dz=0.4, nu=640, nv=480, du=0.6, dv=0.6, n_views=n,
                    theta=full_circle(n), phi=phi, psi=psi, sad=785.0, sdd=1200.0,
                    x_src=x_src, z_src=z_src)


# -- phantoms --------------------------------------------------------------------------

def random_ellipses(seed: int, n: int, r_max: float, axis_range=(4.0, 24.0)):
    """n ellipses (cx, cy, a, b, alpha, density) fully inside the disc of radius r_max."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        a, b = rng.uniform(*axis_range, 2)
        alpha = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.0, 1.0)
        reach = max(a, b)
        rc = max(r_max - reach, 0.0) * math.sqrt(rng.uniform(0.0, 1.0))
        phi = rng.uniform(0.0, 2.0 * math.pi)
        out.append((rc * math.cos(phi), rc * math.sin(phi), a, b, alpha, rho))
    return np.array(out, dtype=np.float64).reshape(n, 6)


def voxelize_ellipses(ell: np.ndarray, nx: int, ny: int, dx: float, dy: float,
                      sub: int = 8) -> np.ndarray:
    """Partial-volume image [ny][nx] (float64) of additive ellipses, sub x sub samples
    per pixel.  Pixel (ix, iy) is centred at ((ix-(nx-1)/2)dx, (iy-(ny-1)/2)dy)."""
    img = np.zeros((ny, nx), dtype=np.float64)
    offs = (np.arange(sub) + 0.5) / sub - 0.5
    for cx, cy, a, b, alpha, rho in ell:
        reach = max(a, b)
        ix0 = max(int(math.floor((cx - reach) / dx + (nx - 1) / 2)) - 1, 0)
        ix1 = min(int(math.ceil((cx + reach) / dx + (nx - 1) / 2)) + 1, nx - 1)
        iy0 = max(int(math.floor((cy - reach) / dy + (ny - 1) / 2)) - 1, 0)
        iy1 = min(int(math.ceil((cy + reach) / dy + (ny - 1) / 2)) + 1, ny - 1)
        if ix1 < ix0 or iy1 < iy0:
            continue
        xs = ((np.arange(ix0, ix1 + 1)[:, None] + offs[None, :]) - (nx - 1) / 2) * dx
        ys = ((np.arange(iy0, iy1 + 1)[:, None] + offs[None, :]) - (ny - 1) / 2) * dy
        X = xs.reshape(1, 1, -1, sub) - cx          # [1,1,NX,s]
        Y = ys.reshape(-1, sub, 1, 1) - cy          # [NY,s,1,1]
        ca, sa = math.cos(alpha), math.sin(alpha)
        p = X * ca + Y * sa
        q = -X * sa + Y * ca
        inside = (p / a) ** 2 + (q / b) ** 2 <= 1.0
        frac = inside.mean(axis=(1, 3))             # [NY, NX]
        img[iy0:iy1 + 1, ix0:ix1 + 1] += rho * frac
    return img


def random_rotation(rng) -> np.ndarray:
    """Uniform random 3x3 rotation from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_ellipsoids(seed: int, n: int, r_max: float, z_max: float,
                      axis_range=(5.0, 30.0)):
    """n ellipsoids as dicts (centre, semi-axes, rotation, density), each inside the
    cylinder r <= r_max, |z| <= z_max."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        axes = rng.uniform(*axis_range, 3)
        rot = random_rotation(rng)
        rho = rng.uniform(0.0, 1.0)
        # half-extents of the rotated ellipsoid along x, y, z
        ext = np.sqrt((rot ** 2) @ (axes ** 2))
        rxy = max(r_max - math.hypot(ext[0], ext[1]), 0.0)
        rc = rxy * math.sqrt(rng.uniform(0.0, 1.0))
        ang = rng.uniform(0.0, 2.0 * math.pi)
        zc = rng.uniform(-1.0, 1.0) * max(z_max - ext[2], 0.0)
        out.append(dict(centre=np.array([rc * math.cos(ang), rc * math.sin(ang), zc]),
                        axes=axes, rot=rot, rho=rho, ext=ext))
    return out


def voxelize_ellipsoids(ells, nx: int, ny: int, nz: int, dx: float, dy: float, dz: float,
                        sub: int = 4) -> np.ndarray:
    """Partial-volume volume [nz][ny][nx] (float64) of additive ellipsoids.

    Each voxel's fraction is the mean over sub x sub lines parallel to z (at the
    sub-pixel centres in x and y) of the exact overlap of the ellipsoid's chord on that
    line with the voxel's z-interval.  Voxel (ix, iy, iz) is centred at
    ((ix-(nx-1)/2)dx, (iy-(ny-1)/2)dy, (iz-(nz-1)/2)dz).
    """
    vol = np.zeros((nz, ny, nx), dtype=np.float64)
    offs = (np.arange(sub) + 0.5) / sub - 0.5
    for e in ells:
        c, axes, rot, rho, ext = e["centre"], e["axes"], e["rot"], e["rho"], e["ext"]
        # quadratic form M = R diag(1/a^2) R^T:  inside <=> (p-c)^T M (p-c) <= 1
        M = rot @ np.diag(1.0 / axes ** 2) @ rot.T
        lo = [int(math.floor((c[k] - ext[k]) / d + (n - 1) / 2)) - 1
              for k, (d, n) in enumerate(((dx, nx), (dy, ny), (dz, nz)))]
        hi = [int(math.ceil((c[k] + ext[k]) / d + (n - 1) / 2)) + 1
              for k, (d, n) in enumerate(((dx, nx), (dy, ny), (dz, nz)))]
        ix0, iy0, iz0 = (max(v, 0) for v in lo)
        ix1, iy1, iz1 = min(hi[0], nx - 1), min(hi[1], ny - 1), min(hi[2], nz - 1)
        if ix1 < ix0 or iy1 < iy0 or iz1 < iz0:
            continue
        xs = (((np.arange(ix0, ix1 + 1)[:, None] + offs[None, :]) - (nx - 1) / 2) * dx
              - c[0]).reshape(-1)
        ys = (((np.arange(iy0, iy1 + 1)[:, None] + offs[None, :]) - (ny - 1) / 2) * dy
              - c[1]).reshape(-1)
        X = xs[None, :]
        Y = ys[:, None]
        # along z: Mzz t^2 + B t + (A - 1) = 0 with t = z - c_z
        A = M[0, 0] * X * X + 2 * M[0, 1] * X * Y + M[1, 1] * Y * Y
        B = 2 * (M[0, 2] * X + M[1, 2] * Y)
        disc = B * B - 4 * M[2, 2] * (A - 1.0)
        root = np.sqrt(np.maximum(disc, 0.0))
        t_lo = np.where(disc > 0, (-B - root) / (2 * M[2, 2]), 0.0) + c[2]
        t_hi = np.where(disc > 0, (-B + root) / (2 * M[2, 2]), 0.0) + c[2]
        zb = ((np.arange(iz0, iz1 + 1) - (nz - 1) / 2) * dz - dz / 2)[:, None, None]
        NY, NX = Y.shape[0] // sub, X.shape[1] // sub
        for k0 in range(0, zb.shape[0], 16):
            zk = zb[k0:k0 + 16]
            ov = np.clip(np.minimum(t_hi[None], zk + dz) - np.maximum(t_lo[None], zk),
                         0.0, None) / dz                      # [Z, NY*s, NX*s]
            frac = ov.reshape(ov.shape[0], NY, sub, NX, sub).mean(axis=(2, 4))
            vol[iz0 + k0:iz0 + k0 + zk.shape[0], iy0:iy1 + 1, ix0:ix1 + 1] += rho * frac
    return vol


def phantom_2d(geom: Geometry, seed: int = 0, n: int = 10, dtype=np.float32) -> np.ndarray:
    """Seeded additive-ellipse image [ny][nx] kept inside the reconstruction circle."""
    r_max = 0.94 * min(geom.nx * geom.dx, geom.ny * geom.dy) / 2.0
    ell = random_ellipses(seed, n, r_max, axis_range=(0.06 * r_max, 0.38 * r_max))
    return voxelize_ellipses(ell, geom.nx, geom.ny, geom.dx, geom.dy).astype(dtype)


def phantom_3d(geom: Geometry, seed: int = 0, n: int = 20, dtype=np.float32,
               sub: int = 4) -> np.ndarray:
    """Seeded additive-ellipsoid volume [nz][ny][nx] kept inside the object cylinder."""
    half_xy = min(geom.nx * geom.dx, geom.ny * geom.dy) / 2.0
    half_z = geom.nz * geom.dz / 2.0
    r_max = 0.94 * half_xy
    z_max = 0.94 * half_z
    s = min(r_max, z_max)
    ells = random_ellipsoids(seed, n, r_max, z_max, axis_range=(0.08 * s, 0.47 * s))
    return voxelize_ellipsoids(ells, geom.nx, geom.ny, geom.nz, geom.dx, geom.dy, geom.dz,
                               sub=sub).astype(dtype)


def phantom(geom: Geometry, seed: int = 0, dtype=np.float32) -> np.ndarray:
    if geom.kind == "fan2d":
        return phantom_2d(geom, seed, dtype=dtype)
    return phantom_3d(geom, seed, dtype=dtype)


def random_volume(geom: Geometry, seed: int = 0, batch: Optional[int] = None,
                  dtype=np.float32) -> np.ndarray:
    """U[0,1) volume(s), shape [batch] + vol_shape."""
    rng = np.random.default_rng(seed)
    shape = geom.vol_shape if batch is None else (batch,) + geom.vol_shape
    return rng.random(shape, dtype=np.float64).astype(dtype)


def random_sinogram(geom: Geometry, seed: int = 0, batch: Optional[int] = None,
                    dtype=np.float32) -> np.ndarray:
    """U[0,1) sinogram(s), shape [batch] + sino_shape."""
    rng = np.random.default_rng(seed + 7919)
    shape = geom.sino_shape if batch is None else (batch,) + geom.sino_shape
    return rng.random(shape, dtype=np.float64).astype(dtype)
