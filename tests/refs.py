"""Independent references used to pin the oracle (no projector footprints here).

* ``cell_rays``: source and detector sub-sample points for every detector cell, written from
  the geometry definition of the paper's Section 2.2 / Table 1 (source at (x_src, SAD, z_src)
  at theta = 0, detector centre at distance SDD, pose R = Rz(theta) Rx(phi) Ry(psi)) with this
  repository's readings (counter-clockwise rotations, e_u = +x and e_v = +z at theta = 0,
  cell centres at (i - (n-1)/2) du - u_ofst).
* ``brute_force``: the detector-cell average of exact line integrals through the voxel grid
  (the exact quantity SF and DD approximate), by S x S sub-rays per cell and the exact
  path-length integrator of ``oracle/exact_ray.c``.
* ``ellipsoid_cell_average``: the same cell average for a continuous ellipsoid phantom, with
  the chord length of each sub-ray through each ellipsoid in closed form.
"""
import math

import numpy as np


def pose(theta, phi=0.0, psi=0.0):
    cz, sz = math.cos(theta), math.sin(theta)
    cx, sx = math.cos(phi), math.sin(phi)
    cy, sy = math.cos(psi), math.sin(psi)
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1.0]])
    Rx = np.array([[1.0, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1.0, 0], [-sy, 0, cy]])
    return Rz @ Rx @ Ry


def cell_rays(geom, view, sub_u, sub_v=1):
    """Segments (a, b) from the source to sub_u x sub_v points inside every detector cell.
    Returns a, b of shape [nv, nu, sub_v, sub_u, 3] (world coordinates relative to the object
    centre, i.e. the object offset is subtracted)."""
    three_d = geom.kind != "fan2d"
    R = pose(geom.per_view("theta")[view],
             geom.per_view("phi")[view] if geom.kind == "cone_noncirc" else 0.0,
             geom.per_view("psi")[view] if geom.kind == "cone_noncirc" else 0.0)
    sad = geom.per_view("sad")[view]
    sdd = geom.per_view("sdd")[view]
    zs = geom.per_view("z_src")[view] if three_d else 0.0
    s = R @ np.array([geom.per_view("x_src")[view], sad, zs])
    d = R @ np.array([0.0, sad - sdd, 0.0])
    eu, ev, n = R @ np.array([1.0, 0, 0]), R @ np.array([0, 0, 1.0]), R @ np.array([0, 1.0, 0])
    o = np.array([geom.per_view("x_ofst")[view], geom.per_view("y_ofst")[view],
                  geom.per_view("z_ofst")[view] if three_d else 0.0])
    nu, nv = geom.nu, (geom.nv if three_d else 1)
    uo = geom.per_view("u_ofst")[view]
    vo = geom.per_view("v_ofst")[view] if three_d else 0.0
    fu = (np.arange(sub_u) + 0.5) / sub_u - 0.5
    fv = (np.arange(sub_v) + 0.5) / sub_v - 0.5 if three_d else np.zeros(1)
    u = ((np.arange(nu) - (nu - 1) / 2)[:, None] + fu[None, :]) * geom.du - uo   # [nu, su]
    if three_d:
        v = ((np.arange(nv) - (nv - 1) / 2)[:, None] + fv[None, :]) * geom.dv - vo
    else:
        v = np.zeros((1, 1))
    U = u[None, :, None, :, None]
    V = v[:, None, :, None, None]
    if geom.det == "flat":
        q = d + U * eu + V * ev
    else:
        gam = U / sdd
        h = V - np.dot(s - d, ev)
        q = s + sdd * (np.sin(gam) * eu - np.cos(gam) * n) + h * ev
    q = q + np.zeros((nv, nu, sub_v if three_d else 1, sub_u, 3))
    a = np.broadcast_to(s, q.shape) - o
    # extend the segment past the detector so the whole object is crossed
    b = a + 1.5 * (q - o - a)
    return np.ascontiguousarray(a), np.ascontiguousarray(b)


def brute_force(orc, geom, vol, views, sub_u=64, sub_v=16):
    """Cell-averaged exact line integrals [len(views)][nv][nu] (2D: [len(views)][nu])."""
    three_d = geom.kind != "fan2d"
    v3 = vol if three_d else vol[None]
    nz = geom.nz if three_d else 1
    out = []
    for view in views:
        a, b = cell_rays(geom, view, sub_u, sub_v if three_d else 1)
        shp = a.shape[:-1]
        vals = orc.ray_integrals(v3, (geom.nx, geom.ny, nz),
                                 (geom.dx, geom.dy, geom.dz if three_d else 1.0),
                                 (0.0, 0.0, 0.0), a.reshape(-1, 3), b.reshape(-1, 3))
        vals = vals.reshape(shp).mean(axis=(2, 3))      # [nv, nu]
        out.append(vals if three_d else vals[0])
    return np.stack(out)


def ellipsoid_chords(a, b, centre, axes, rot):
    """Length of segment a->b (arrays [..., 3]) inside the ellipsoid {p: |D R^T (p-c)| <= 1}."""
    Dinv = 1.0 / np.asarray(axes)
    pa = ((a - centre) @ rot) * Dinv
    dirv = ((b - a) @ rot) * Dinv
    A = np.sum(dirv * dirv, axis=-1)
    B = 2 * np.sum(pa * dirv, axis=-1)
    C = np.sum(pa * pa, axis=-1) - 1.0
    disc = B * B - 4 * A * C
    root = np.sqrt(np.maximum(disc, 0.0))
    t0 = np.clip((-B - root) / (2 * A), 0.0, 1.0)
    t1 = np.clip((-B + root) / (2 * A), 0.0, 1.0)
    seg = np.linalg.norm(b - a, axis=-1)
    return np.where(disc > 0, (t1 - t0) * seg, 0.0)


def ellipsoid_cell_average(geom, ells, views, sub_u=8, sub_v=8):
    """Cell-averaged analytic line integrals of additive ellipsoids [len(views)][nv][nu]."""
    out = []
    for view in views:
        a, b = cell_rays(geom, view, sub_u, sub_v)
        acc = np.zeros(a.shape[:-1])
        for e in ells:
            acc += e["rho"] * ellipsoid_chords(a, b, e["centre"], e["axes"], e["rot"])
        out.append(acc.mean(axis=(2, 3)))
    return np.stack(out)


def _frame(geom, view):
    three_d = geom.kind != "fan2d"
    R = pose(geom.per_view("theta")[view],
             geom.per_view("phi")[view] if geom.kind == "cone_noncirc" else 0.0,
             geom.per_view("psi")[view] if geom.kind == "cone_noncirc" else 0.0)
    sad, sdd = geom.per_view("sad")[view], geom.per_view("sdd")[view]
    zs = geom.per_view("z_src")[view] if three_d else 0.0
    s = R @ np.array([geom.per_view("x_src")[view], sad, zs])
    d = R @ np.array([0.0, sad - sdd, 0.0])
    return s, d, R @ np.array([1.0, 0, 0]), R @ np.array([0, 0, 1.0]), R @ np.array([0, 1.0, 0])


def piecewise_exact(orc, geom, vol, view):
    """Cell averages of exact line integrals for a flat detector, integrated exactly when the
    integral is piecewise polynomial of low degree in (u, v) between the detector positions
    of the voxel corners -- which holds for parallel rays.  Each cell is cut at every corner
    position that falls inside it and each piece gets 2-point Gauss-Legendre nodes per axis
    (exact for bilinear pieces); the rays through the nodes are integrated exactly.
    Returns [nv][nu] (2D: [nu])."""
    assert geom.det == "flat"
    three_d = geom.kind != "fan2d"
    s, d, eu, ev, n = _frame(geom, view)
    nz = geom.nz if three_d else 1
    xs = (np.arange(geom.nx + 1) - geom.nx / 2) * geom.dx
    ys = (np.arange(geom.ny + 1) - geom.ny / 2) * geom.dy
    zs = (np.arange(nz + 1) - nz / 2) * geom.dz if three_d else np.zeros(1)
    P = np.stack(np.meshgrid(xs, ys, zs, indexing="ij"), -1).reshape(-1, 3)
    D = np.dot(s - d, n)
    W = np.dot(s - P, n)
    ub = np.dot(s - d, eu) + D * ((P - s) @ eu) / W
    vb = np.dot(s - d, ev) + D * ((P - s) @ ev) / W
    uo = geom.per_view("u_ofst")[view]
    vo = geom.per_view("v_ofst")[view] if three_d else 0.0
    ue = (np.arange(geom.nu + 1) - geom.nu / 2) * geom.du - uo
    nv = geom.nv if three_d else 1
    ve = (np.arange(nv + 1) - nv / 2) * geom.dv - vo if three_d else np.array([-0.5, 0.5])
    gl = np.array([-1.0, 1.0]) / math.sqrt(3.0)

    def nodes(lo, hi, brk):
        cuts = np.unique(np.concatenate([[lo, hi], brk[(brk > lo) & (brk < hi)]]))
        a, b = cuts[:-1], cuts[1:]
        x = (0.5 * (a + b))[:, None] + (0.5 * (b - a))[:, None] * gl[None, :]
        w = np.repeat(0.5 * (b - a), 2) / (hi - lo)
        return x.reshape(-1), w

    out = np.zeros((nv, geom.nu))
    vol3 = vol if three_d else vol[None]
    for j in range(nv):
        vn, vw = nodes(ve[j], ve[j + 1], vb) if three_d else (np.zeros(1), np.ones(1))
        for i in range(geom.nu):
            un, uw = nodes(ue[i], ue[i + 1], ub)
            U, V = np.meshgrid(un, vn, indexing="xy")
            q = d + U[..., None] * eu + V[..., None] * ev
            a = np.broadcast_to(s, q.shape)
            b = a + 1.5 * (q - a)
            val = orc.ray_integrals(vol3, (geom.nx, geom.ny, nz),
                                    (geom.dx, geom.dy, geom.dz if three_d else 1.0),
                                    (0.0, 0.0, 0.0), a.reshape(-1, 3), b.reshape(-1, 3))
            out[j, i] = np.sum(val.reshape(U.shape) * (vw[:, None] * uw[None, :]))
    return out if three_d else out[0]
