"""FP64 ramp filtering for filtered back projection -- TEST INFRASTRUCTURE ONLY (see the
package docstring: only the tests, the smoke check and the benchmark's CPU leg use it).

The paper ships a discrete ramp filter and a "recon" projector mode whose back projection
carries the depth weight of FBP (Section 2.1 and 2.3, citing Kak and Slaney).  Written here
from the textbook fan-beam formulas on the real detector:

  flat detector (equally spaced cells):
      q_i = dbeta * (M du / 2) * sum_k h(i - k) c_k p_k,   M = SDD / SAD,
      c_k = SDD / sqrt(SDD^2 + (u_k - x_src)^2 + (v_j - z_src)^2)   (2D: no v term),
  curved detector (equiangular, gamma = u / SDD, dgamma = du / SDD):
      q_i = dbeta * (dgamma / (2 SAD)) * sum_k (g/sin g)^2 h(i - k) c_k p_k,  g = (i - k) dgamma,
      c_k = cos(gamma_k) * SDD / sqrt(SDD^2 + (v_j - z_src)^2),
with h the band-limited ramp sampled at the cell pitch a (du, or dgamma):
  Ram-Lak:     h(0) = 1/(4 a^2), h(n) = 0 (n even), -1/(n^2 pi^2 a^2) (n odd);
  Shepp-Logan: h(n) = -2 / (pi^2 a^2 (4 n^2 - 1)),
and dbeta = 2 pi / n_views (a full circular scan, uniformly sampled).  The reconstruction is
then the "recon"-mode back projection sum_b (SAD/W)^2 (normalised footprint) q_b.
"""
from __future__ import annotations

import numpy as np

WINDOWS = ("ram-lak", "shepp-logan")


def ramp_taps(n: int, a: float, window: str = "ram-lak") -> np.ndarray:
    """h(k a) for k = -(n-1) .. n-1."""
    k = np.arange(-(n - 1), n, dtype=np.float64)
    if window == "ram-lak":
        h = np.zeros_like(k)
        h[k == 0] = 1.0 / (4.0 * a * a)
        odd = (np.abs(k) % 2) == 1
        h[odd] = -1.0 / (np.pi ** 2 * k[odd] ** 2 * a * a)
        return h
    if window == "shepp-logan":
        return -2.0 / (np.pi ** 2 * a * a * (4.0 * k * k - 1.0))
    raise ValueError(f"unknown window {window!r}")


def _cols(geom):
    return (np.arange(geom.nu) - (geom.nu - 1) / 2.0) * geom.du


def ramp_filter(geom, sino, window: str = "ram-lak") -> np.ndarray:
    """Cosine-weight, ramp-filter and scale a sinogram (sino_shape, or [B] + sino_shape) for
    FBP / FDK on a circular scan.  Returns float64 of the same shape."""
    p = np.asarray(sino, dtype=np.float64)
    two_d = geom.kind == "fan2d"
    if geom.kind == "cone_noncirc":
        raise NotImplementedError("FBP weighting is defined for circular scans")
    nu, nb = geom.nu, geom.n_views
    view_shape = (nu,) if two_d else (geom.nv, nu)
    batched = p.ndim == len(geom.sino_shape) + 1
    ps = p if batched else p[None]
    out = np.zeros_like(ps)
    dbeta = 2.0 * np.pi / nb
    idx = np.arange(nu)
    diff = idx[:, None] - idx[None, :]                      # i - k
    for b in range(nb):
        sad = float(geom.per_view("sad")[b])
        sdd = float(geom.per_view("sdd")[b])
        u = _cols(geom) - float(geom.per_view("u_ofst")[b])
        if two_d:
            v = np.zeros(1)
        else:
            v = (np.arange(geom.nv) - (geom.nv - 1) / 2.0) * geom.dv - float(geom.per_view("v_ofst")[b])
        zs = 0.0 if two_d else float(geom.per_view("z_src")[b])
        if geom.det == "flat":
            xs = float(geom.per_view("x_src")[b])
            taps = ramp_taps(nu, geom.du, window)
            H = taps[diff + nu - 1] * (sdd / sad) * geom.du / 2.0
            c = sdd / np.sqrt(sdd ** 2 + (u[None, :] - xs) ** 2 + (v[:, None] - zs) ** 2)
        else:
            dg = geom.du / sdd
            taps = ramp_taps(nu, dg, window)
            g = diff * dg
            ratio = np.ones_like(g)
            nz = diff != 0
            ratio[nz] = (g[nz] / np.sin(g[nz])) ** 2
            H = taps[diff + nu - 1] * ratio * dg / (2.0 * sad)
            c = np.cos(u[None, :] / sdd) * sdd / np.sqrt(sdd ** 2 + (v[:, None] - zs) ** 2)
        for it in range(ps.shape[0]):
            rows = ps[it, b].reshape((-1, nu)) * c             # [rows][nu]
            out[it, b] = (dbeta * rows @ H.T).reshape(view_shape)
    return out if batched else out[0]
