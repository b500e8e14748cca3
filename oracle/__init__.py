"""FP64 CPU oracle for the SF / DD projectors -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The product path (the HIP engine and its binding) never imports,
links or calls it, and it imports nothing from the engine: the two meet only through the
seeded inputs of ``paper_2503_16741_amd.synth``.

Functions follow the paper's Eq. 1 (forward, y = A x) and Eq. 2 (adjoint, x = A^T y);
``ctoracle.c`` documents each step.  ``exact_ray.c`` is an independent brute-force
reference (exact path lengths through the voxel grid) used only to pin the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libctoracle.so")
_SOURCES = ("ctoracle.c", "exact_ray.c")
_lib = None

METHODS = {"sf": 0, "dd": 1}
MODES = ("proj", "recon")
KIND = {"fan2d": 0, "cone": 1, "cone_noncirc": 2}
DET = {"flat": 0, "curved": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH) and all(
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(s) for s in srcs):
        return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Geom(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("det", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("n_views", ctypes.c_int32)] + [
        (name, ctypes.POINTER(ctypes.c_double)) for name in
        ("theta", "phi", "psi", "sad", "sdd", "x_src", "z_src",
         "x_ofst", "y_ofst", "z_ofst", "u_ofst", "v_ofst")]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = load(_LIB_PATH)
    return _lib


def load(path: str):
    """The oracle library at `path` with its entry points typed (the test suite also loads
    deliberately broken builds of it, to show that the pins catch them)."""
    L = ctypes.CDLL(path)
    L.orc_forward.restype = ctypes.c_int
    L.orc_forward.argtypes = [ctypes.POINTER(_Geom), ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_adjoint.restype = ctypes.c_int
    L.orc_adjoint.argtypes = [ctypes.POINTER(_Geom), ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_count.restype = ctypes.c_int
    L.orc_count.argtypes = [ctypes.POINTER(_Geom), ctypes.c_int, ctypes.c_int,
                            ctypes.c_void_p, ctypes.c_void_p]
    L.orc_num_threads.restype = ctypes.c_int
    L.exr_integrals.restype = ctypes.c_int
    L.exr_integrals.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64] + [ctypes.c_void_p] * 3
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cgeom(geom):
    """ctypes geometry with every per-view parameter broadcast to n_views doubles."""
    keep = {}
    g = _Geom()
    g.kind, g.det = KIND[geom.kind], DET[geom.det]
    two_d = geom.kind == "fan2d"
    g.nx, g.ny, g.nz = geom.nx, geom.ny, 1 if two_d else geom.nz
    g.dx, g.dy, g.dz = geom.dx, geom.dy, geom.dz
    g.nu, g.nv = geom.nu, 1 if two_d else geom.nv
    g.du, g.dv = geom.du, geom.dv
    g.n_views = geom.n_views
    for name in ("theta", "phi", "psi", "sad", "sdd", "x_src", "z_src",
                 "x_ofst", "y_ofst", "z_ofst", "u_ofst", "v_ofst"):
        arr = np.ascontiguousarray(geom.per_view(name), dtype=np.float64)
        keep[name] = arr
        setattr(g, name, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return g, keep


def _code(method: str, mode: str) -> int:
    """Oracle method code: 0 = SF, 1 = DD, 2 = SF in "recon" mode (FBP weighting)."""
    if mode not in MODES:
        raise ValueError(f"mode must be one of {MODES}")
    if mode == "recon":
        if method != "sf":
            raise NotImplementedError("recon mode is defined for the SF projector")
        return 2
    return METHODS[method]


def _check(rc):
    if rc == -2:
        raise NotImplementedError("geometry/method combination not defined by the oracle")
    if rc != 0:
        raise ValueError(f"oracle error {rc}")


def forward(geom, vol, method: str = "sf", views=None, mode: str = "proj") -> np.ndarray:
    """y = A x for the listed views (default: all).  vol: vol_shape (or [B] + vol_shape).
    Returns float64 [len(views)][nv][nu] (2D: [len(views)][nu]), with a leading batch
    axis when vol has one.  mode "recon": the transpose of the FBP back projection."""
    vol = np.asarray(vol)
    batched = vol.ndim == len(geom.vol_shape) + 1
    vols = vol if batched else vol[None]
    views = np.arange(geom.n_views, dtype=np.int32) if views is None else \
        np.ascontiguousarray(np.asarray(views, dtype=np.int32).reshape(-1))
    g, keep = _cgeom(geom)
    nv = 1 if geom.kind == "fan2d" else geom.nv
    outs = []
    for v in vols:
        v64 = np.ascontiguousarray(v, dtype=np.float64)
        out = np.zeros((views.size, nv, geom.nu), dtype=np.float64)
        _check(lib().orc_forward(ctypes.byref(g), _code(method, mode), _ptr(v64), int(views.size),
                                 _ptr(views), _ptr(out)))
        outs.append(out.reshape((views.size, geom.nu)) if geom.kind == "fan2d" else out)
    del keep
    return np.stack(outs) if batched else outs[0]


def adjoint(geom, sino, method: str = "sf", voxels=None, mode: str = "proj") -> np.ndarray:
    """x = A^T y.  sino: sino_shape (or [B] + sino_shape).  With voxels=None returns the full
    volume (vol_shape); otherwise the values at the given linear voxel indices.  mode "recon":
    the FBP back projection sum_b (SAD/W)^2 (normalised SF footprint) y_b."""
    sino = np.asarray(sino)
    batched = sino.ndim == len(geom.sino_shape) + 1
    sinos = sino if batched else sino[None]
    full = voxels is None
    idx = np.arange(geom.n_vox, dtype=np.int64) if full else \
        np.ascontiguousarray(np.asarray(voxels, dtype=np.int64).reshape(-1))
    g, keep = _cgeom(geom)
    outs = []
    for s in sinos:
        s64 = np.ascontiguousarray(s, dtype=np.float64)
        out = np.zeros(idx.size, dtype=np.float64)
        _check(lib().orc_adjoint(ctypes.byref(g), _code(method, mode), _ptr(s64), int(idx.size),
                                 _ptr(idx), _ptr(out)))
        outs.append(out.reshape(geom.vol_shape) if full else out)
    del keep
    return np.stack(outs) if batched else outs[0]


def count(geom, method: str = "sf", views=None) -> dict:
    """Footprint statistics over the listed views: voxel-views that reach the detector,
    non-zeros of A, touched columns and touched rows (summed over voxel-views)."""
    views = np.arange(geom.n_views, dtype=np.int32) if views is None else \
        np.ascontiguousarray(np.asarray(views, dtype=np.int32).reshape(-1))
    g, keep = _cgeom(geom)
    out = np.zeros(4, dtype=np.int64)
    _check(lib().orc_count(ctypes.byref(g), METHODS[method], int(views.size), _ptr(views),
                           _ptr(out)))
    del keep
    return dict(voxel_views=int(out[0]), nnz=int(out[1]), cols=int(out[2]), rows=int(out[3]))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def ray_integrals(vol, shape_xyz, pitch_xyz, origin_xyz, a, b) -> np.ndarray:
    """Exact line integrals of the voxel grid along segments a[r] -> b[r] (brute force).
    vol is [nz][ny][nx]; shape/pitch/origin are (x, y, z) triples; the grid is centred at
    origin."""
    v64 = np.ascontiguousarray(vol, dtype=np.float64)
    n = np.ascontiguousarray(shape_xyz, dtype=np.int32)
    h = np.ascontiguousarray(pitch_xyz, dtype=np.float64)
    o = np.ascontiguousarray(origin_xyz, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(a.shape[0], dtype=np.float64)
    lib().exr_integrals(_ptr(v64), _ptr(n), _ptr(h), _ptr(o), int(a.shape[0]), _ptr(a),
                        _ptr(b), _ptr(out))
    return out


def fbp(geom, sino, window: str = "ram-lak", voxels=None) -> np.ndarray:
    """Filtered back projection (fan beam) / FDK (cone beam) of a circular scan: the ramp
    filter of ``ramp.py`` followed by the "recon"-mode back projection."""
    from .ramp import ramp_filter
    return adjoint(geom, ramp_filter(geom, sino, window), voxels=voxels, mode="recon")
