"""ctypes binding of ``libctproj.so`` (include/ctproj.h).

Argument marshalling only: every step of the projection runs in the library's HIP kernels.
The functions keep the C names; ``Plan`` owns a plan handle and frees it on ``close()``.
Tensors passed in must be contiguous CUDA (HIP) tensors of float32, bfloat16 or float16 (the
storage type; arithmetic is always FP32); the current torch stream
is used unless one is given.  If the library is not built the first call raises -- there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional

import numpy as np

from .synth import Geometry, PER_VIEW

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctproj.so")

CTP_OK, CTP_EINVAL, CTP_EUNSUPPORTED, CTP_ENOMEM, CTP_EDEVICE = 0, -1, -2, -3, -4
CTP_FAN2D, CTP_CONE_CIRC, CTP_CONE_NONCIRC = 0, 1, 2
CTP_DET_FLAT, CTP_DET_CURVED = 0, 1
CTP_SF, CTP_DD = 0, 1
CTP_F32, CTP_BF16, CTP_F16 = 0, 1, 2
CTP_FORWARD, CTP_BACKWARD = 0, 1

KIND = {"fan2d": CTP_FAN2D, "cone": CTP_CONE_CIRC, "cone_noncirc": CTP_CONE_NONCIRC}
DET = {"flat": CTP_DET_FLAT, "curved": CTP_DET_CURVED}
METHOD = {"sf": CTP_SF, "dd": CTP_DD}

EXPORTED = ("ctp_plan_create", "ctp_plan_destroy", "ctp_plan_bytes", "ctp_workspace_bytes",
            "ctp_project", "ctp_backproject", "ctp_status_string", "ctp_last_error")


class CtpError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {_status_name(status)} ({status}): {detail}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = ([("kind", ctypes.c_int), ("det", ctypes.c_int),
                 ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                 ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                 ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                 ("du", ctypes.c_double), ("dv", ctypes.c_double),
                 ("n_views", ctypes.c_int32)]
                + [(n, ctypes.POINTER(ctypes.c_double)) for n in PER_VIEW]
                + [("len_" + n, ctypes.c_int32) for n in PER_VIEW])


_lib = None
_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """Open libctproj.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with `python paper_2503_16741_amd/build.py` "
                    "(or __graft_entry__.build()); there is no CPU fallback")
            L = ctypes.CDLL(LIB_PATH)
            vp, sz, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
            L.ctp_plan_create.argtypes = [ctypes.POINTER(_Desc), ctypes.c_int, ctypes.POINTER(vp)]
            L.ctp_plan_destroy.argtypes = [vp]
            L.ctp_plan_bytes.argtypes = [vp, ctypes.c_int, i64, ctypes.POINTER(sz), ctypes.POINTER(sz)]
            L.ctp_workspace_bytes.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, i64,
                                              ctypes.POINTER(sz)]
            L.ctp_project.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, i64, ctypes.c_int,
                                      vp, sz, vp]
            L.ctp_backproject.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, i64, ctypes.c_int,
                                          vp, sz, vp]
            for f in ("ctp_plan_create", "ctp_plan_destroy", "ctp_plan_bytes",
                      "ctp_workspace_bytes", "ctp_project", "ctp_backproject"):
                getattr(L, f).restype = ctypes.c_int
            L.ctp_status_string.argtypes = [ctypes.c_int]
            L.ctp_status_string.restype = ctypes.c_char_p
            L.ctp_last_error.argtypes = []
            L.ctp_last_error.restype = ctypes.c_char_p
            _lib = L
    return _lib


def _status_name(st: int) -> str:
    try:
        return lib().ctp_status_string(st).decode()
    except Exception:  # noqa: BLE001 - only used to format an error
        return str(st)


def ctp_status_string(status: int) -> str:
    return lib().ctp_status_string(status).decode()


def ctp_last_error() -> str:
    return lib().ctp_last_error().decode()


def _check(st: int, where: str):
    if st != CTP_OK:
        raise CtpError(st, where, ctp_last_error())


class Plan:
    """Owner of a ``ctp_plan*`` plus the geometry it was built from."""

    def __init__(self, handle: int, geom: Geometry, method: str):
        self.handle = ctypes.c_void_p(handle)
        self.geom = geom
        self.method = method
        self._ws = {}

    def close(self):
        if self.handle:
            ctp_plan_destroy(self)

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def make_desc(geom: Geometry):
    """Fill the C descriptor; returns (desc, keep-alive arrays)."""
    d = _Desc()
    d.kind, d.det = KIND[geom.kind], DET[geom.det]
    two_d = geom.kind == "fan2d"
    d.nx, d.ny, d.nz = geom.nx, geom.ny, 1 if two_d else geom.nz
    d.dx, d.dy, d.dz = geom.dx, geom.dy, geom.dz
    d.nu, d.nv = geom.nu, 1 if two_d else geom.nv
    d.du, d.dv = geom.du, geom.dv
    d.n_views = geom.n_views
    keep = []
    for name in PER_VIEW:
        arr = np.ascontiguousarray(geom.param(name), dtype=np.float64)
        keep.append(arr)
        setattr(d, name, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        setattr(d, "len_" + name, int(arr.size))
    return d, keep


def ctp_plan_create(geom: Geometry, method: str = "sf") -> Plan:
    d, keep = make_desc(geom)
    out = ctypes.c_void_p()
    _check(lib().ctp_plan_create(ctypes.byref(d), METHOD[method], ctypes.byref(out)),
           "ctp_plan_create")
    del keep
    return Plan(out.value, geom, method)


def ctp_plan_destroy(plan: Plan):
    h, plan.handle = plan.handle, ctypes.c_void_p()
    plan._ws.clear()
    _check(lib().ctp_plan_destroy(h), "ctp_plan_destroy")


def ctp_plan_bytes(plan: Plan, batch: int = 1, dtype: int = CTP_F32):
    vb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().ctp_plan_bytes(plan.handle, dtype, batch, ctypes.byref(vb), ctypes.byref(sb)),
           "ctp_plan_bytes")
    return vb.value, sb.value


def ctp_workspace_bytes(plan: Plan, direction: int, batch: int = 1, vol_dtype: int = CTP_F32,
                        sino_dtype: int = CTP_F32) -> int:
    b = ctypes.c_size_t()
    _check(lib().ctp_workspace_bytes(plan.handle, direction, vol_dtype, sino_dtype, batch,
                                     ctypes.byref(b)), "ctp_workspace_bytes")
    return b.value


def _dtype_code(t) -> int:
    import torch
    codes = {torch.float32: CTP_F32, torch.bfloat16: CTP_BF16, torch.float16: CTP_F16}
    if t.dtype not in codes:
        raise TypeError(f"unsupported dtype {t.dtype}: use float32, bfloat16 or float16")
    return codes[t.dtype]


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _workspace(plan: Plan, direction: int, batch: int, device, vol_dtype=CTP_F32,
               sino_dtype=CTP_F32):
    """A cached, 256-byte-aligned workspace tensor for this plan/direction/batch (torch
    allocations are 512-byte aligned)."""
    import torch
    need = ctp_workspace_bytes(plan, direction, batch, vol_dtype, sino_dtype)
    if need == 0:
        return None, 0
    key = (direction, str(device))
    ws = plan._ws.get(key)
    if ws is None or ws.numel() * 4 < need:
        ws = torch.empty((need + 3) // 4, dtype=torch.float32, device=device)
        plan._ws[key] = ws
    return ws, need


def _check_tensor(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    _dtype_code(t)
    if tuple(t.shape[-len(shape):]) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [...]+{tuple(shape)}")


def ctp_project(plan: Plan, vol, sino, accumulate: bool = False, workspace=None,
                stream=None):
    """sino (+)= A vol on the device.  vol: [B]+vol_shape, sino: [B]+sino_shape."""
    g = plan.geom
    _check_tensor(vol, g.vol_shape, "vol")
    _check_tensor(sino, g.sino_shape, "sino")
    batch = vol.numel() // int(np.prod(g.vol_shape))
    if sino.numel() != batch * int(np.prod(g.sino_shape)):
        raise ValueError("vol and sino batch sizes differ")
    vd, sd = _dtype_code(vol), _dtype_code(sino)
    if workspace is None:
        ws, nbytes = _workspace(plan, CTP_FORWARD, batch, vol.device, vd, sd)
    else:
        ws, nbytes = workspace, workspace.numel() * workspace.element_size()
    _check(lib().ctp_project(plan.handle, vol.data_ptr(), vd, sino.data_ptr(), sd,
                             batch, int(bool(accumulate)),
                             ws.data_ptr() if ws is not None else None, nbytes,
                             _stream_handle(stream)), "ctp_project")
    return sino


def ctp_backproject(plan: Plan, sino, vol, accumulate: bool = False, workspace=None,
                    stream=None):
    """vol (+)= A^T sino on the device."""
    g = plan.geom
    _check_tensor(vol, g.vol_shape, "vol")
    _check_tensor(sino, g.sino_shape, "sino")
    batch = vol.numel() // int(np.prod(g.vol_shape))
    if sino.numel() != batch * int(np.prod(g.sino_shape)):
        raise ValueError("vol and sino batch sizes differ")
    vd, sd = _dtype_code(vol), _dtype_code(sino)
    if workspace is None:
        ws, nbytes = _workspace(plan, CTP_BACKWARD, batch, vol.device, vd, sd)
    else:
        ws, nbytes = workspace, workspace.numel() * workspace.element_size()
    _check(lib().ctp_backproject(plan.handle, sino.data_ptr(), sd, vol.data_ptr(), vd,
                                 batch, int(bool(accumulate)),
                                 ws.data_ptr() if ws is not None else None, nbytes,
                                 _stream_handle(stream)), "ctp_backproject")
    return vol


def project(plan: Plan, vol, out_dtype=None):
    """Convenience: allocate the sinogram (same storage type as vol unless given) and
    forward-project."""
    import torch
    g = plan.geom
    lead = tuple(vol.shape[:vol.dim() - len(g.vol_shape)])
    sino = torch.empty(lead + tuple(g.sino_shape), dtype=out_dtype or vol.dtype, device=vol.device)
    return ctp_project(plan, vol, sino)


def backproject(plan: Plan, sino, out_dtype=None):
    """Convenience: allocate the volume (same storage type as sino unless given) and
    back-project."""
    import torch
    g = plan.geom
    lead = tuple(sino.shape[:sino.dim() - len(g.sino_shape)])
    vol = torch.empty(lead + tuple(g.vol_shape), dtype=out_dtype or sino.dtype, device=sino.device)
    return ctp_backproject(plan, sino, vol)
