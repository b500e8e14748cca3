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

CTP_OK, CTP_EINVAL, CTP_EUNSUPPORTED, CTP_ENOMEM, CTP_EDEVICE, CTP_ETIMEOUT = 0, -1, -2, -3, -4, -5
CTP_ECANCELED = -6
CTP_FAN2D, CTP_CONE_CIRC, CTP_CONE_NONCIRC = 0, 1, 2
CTP_DET_FLAT, CTP_DET_CURVED = 0, 1
CTP_SF, CTP_DD = 0, 1
CTP_F32, CTP_BF16, CTP_F16 = 0, 1, 2
CTP_FORWARD, CTP_BACKWARD = 0, 1
CTP_MODE_PROJ, CTP_MODE_RECON = 0, 1
CTP_WINDOW_RAMLAK, CTP_WINDOW_SHEPP_LOGAN = 0, 1

KIND = {"fan2d": CTP_FAN2D, "cone": CTP_CONE_CIRC, "cone_noncirc": CTP_CONE_NONCIRC}
DET = {"flat": CTP_DET_FLAT, "curved": CTP_DET_CURVED}
METHOD = {"sf": CTP_SF, "dd": CTP_DD}
MODE = {"proj": CTP_MODE_PROJ, "recon": CTP_MODE_RECON}
WINDOW = {"ram-lak": CTP_WINDOW_RAMLAK, "shepp-logan": CTP_WINDOW_SHEPP_LOGAN}

EXPORTED = ("ctp_plan_create", "ctp_plan_destroy", "ctp_plan_bytes", "ctp_workspace_bytes",
            "ctp_project", "ctp_project_static", "ctp_backproject", "ctp_ramp_filter",
            "ctp_status_string", "ctp_last_error")
# include/ctserve.h
EXPORTED_SERVER = ("ctp_server_create", "ctp_server_submit", "ctp_server_wait",
                   "ctp_server_query", "ctp_server_info", "ctp_server_cancel",
                   "ctp_server_release", "ctp_server_get_stats", "ctp_server_destroy")


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


class _ServerConfig(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("n_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("age_cap_us", ctypes.c_int64), ("express_work", ctypes.c_double),
                ("launch_work", ctypes.c_double)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("batch", ctypes.c_int32), ("slot", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("calls", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("max_running", ctypes.c_int32), ("max_batch_seen", ctypes.c_int32),
                ("arena_peak", ctypes.c_size_t)]


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
            L.ctp_plan_create.argtypes = [ctypes.POINTER(_Desc), ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(vp)]
            L.ctp_ramp_filter.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, i64, ctypes.c_int,
                                          vp]
            L.ctp_plan_destroy.argtypes = [vp]
            L.ctp_plan_bytes.argtypes = [vp, ctypes.c_int, i64, ctypes.POINTER(sz), ctypes.POINTER(sz)]
            L.ctp_workspace_bytes.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, i64,
                                              ctypes.POINTER(sz)]
            L.ctp_project.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, i64, ctypes.c_int,
                                      vp, sz, vp]
            L.ctp_backproject.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, i64, ctypes.c_int,
                                          vp, sz, vp]
            L.ctp_project_static.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, i64,
                                             ctypes.c_int, vp]
            for f in ("ctp_plan_create", "ctp_plan_destroy", "ctp_plan_bytes",
                      "ctp_workspace_bytes", "ctp_project", "ctp_project_static",
                      "ctp_backproject", "ctp_ramp_filter"):
                getattr(L, f).restype = ctypes.c_int
            u64 = ctypes.c_uint64
            L.ctp_server_create.argtypes = [ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]
            L.ctp_server_submit.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int,
                                            vp, ctypes.POINTER(u64)]
            L.ctp_server_wait.argtypes = [vp, u64, i64, ctypes.POINTER(vp)]
            L.ctp_server_query.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(vp)]
            L.ctp_server_info.argtypes = [vp, u64, ctypes.POINTER(_RequestInfo)]
            L.ctp_server_cancel.argtypes = [vp, u64]
            L.ctp_server_release.argtypes = [vp, u64, vp]
            L.ctp_server_get_stats.argtypes = [vp, ctypes.POINTER(_ServerStats)]
            L.ctp_server_destroy.argtypes = [vp]
            for f in EXPORTED_SERVER:
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

    def __init__(self, handle: int, geom: Geometry, method: str, mode: str = "proj"):
        self.handle = ctypes.c_void_p(handle)
        self.geom = geom
        self.method = method
        self.mode = mode
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


def ctp_plan_create(geom: Geometry, method: str = "sf", mode: str = "proj") -> Plan:
    d, keep = make_desc(geom)
    out = ctypes.c_void_p()
    _check(lib().ctp_plan_create(ctypes.byref(d), METHOD[method], MODE[mode], ctypes.byref(out)),
           "ctp_plan_create")
    del keep
    return Plan(out.value, geom, method, mode)


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
    allocations are 512-byte aligned).  One cache entry per plan, direction and device: calls
    that use the default workspace of the same plan must not run concurrently on different
    streams (pass ``workspace=`` for that)."""
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


def _default_workspace(plan: Plan, direction: int, batch: int, device, vd, sd, stream):
    """The cached workspace for a call on `stream`.  When the call runs on another stream than
    the current one, the caching allocator is told (record_stream), so that the block is not
    handed to a new allocation while that call may still use it; a raw stream handle gives the
    allocator nothing to track, so it needs an explicit workspace."""
    ws, nbytes = _workspace(plan, direction, batch, device, vd, sd)
    if ws is not None and stream is not None:
        if not hasattr(stream, "cuda_stream"):
            raise ValueError("pass workspace= with a raw stream handle")
        ws.record_stream(stream)
    return ws, nbytes


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
        ws, nbytes = _default_workspace(plan, CTP_FORWARD, batch, vol.device, vd, sd, stream)
    else:
        ws, nbytes = workspace, workspace.numel() * workspace.element_size()
    _check(lib().ctp_project(plan.handle, vol.data_ptr(), vd, sino.data_ptr(), sd,
                             batch, int(bool(accumulate)),
                             ws.data_ptr() if ws is not None else None, nbytes,
                             _stream_handle(stream)), "ctp_project")
    return sino


def ctp_project_static(plan: Plan, vol, sino, accumulate: bool = False, stream=None):
    """sino (+)= A vol using the library's static per-device scratch (no allocation; calls on
    one device must not overlap)."""
    g = plan.geom
    _check_tensor(vol, g.vol_shape, "vol")
    _check_tensor(sino, g.sino_shape, "sino")
    batch = vol.numel() // int(np.prod(g.vol_shape))
    if sino.numel() != batch * int(np.prod(g.sino_shape)):
        raise ValueError("vol and sino batch sizes differ")
    _check(lib().ctp_project_static(plan.handle, vol.data_ptr(), _dtype_code(vol), sino.data_ptr(),
                                    _dtype_code(sino), batch, int(bool(accumulate)),
                                    _stream_handle(stream)), "ctp_project_static")
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
        ws, nbytes = _default_workspace(plan, CTP_BACKWARD, batch, vol.device, vd, sd, stream)
    else:
        ws, nbytes = workspace, workspace.numel() * workspace.element_size()
    _check(lib().ctp_backproject(plan.handle, sino.data_ptr(), sd, vol.data_ptr(), vd,
                                 batch, int(bool(accumulate)),
                                 ws.data_ptr() if ws is not None else None, nbytes,
                                 _stream_handle(stream)), "ctp_backproject")
    return vol


def ctp_ramp_filter(plan: Plan, sino, out, window: str = "ram-lak", stream=None):
    """out = cosine-weighted, ramp-filtered sino (FBP / FDK weighting of a full circular scan);
    out may be sino itself when the storage types agree."""
    g = plan.geom
    _check_tensor(sino, g.sino_shape, "sino")
    _check_tensor(out, g.sino_shape, "out")
    batch = sino.numel() // int(np.prod(g.sino_shape))
    if out.numel() != sino.numel():
        raise ValueError("sino and out sizes differ")
    _check(lib().ctp_ramp_filter(plan.handle, sino.data_ptr(), _dtype_code(sino), out.data_ptr(),
                                 _dtype_code(out), batch, WINDOW[window], _stream_handle(stream)),
           "ctp_ramp_filter")
    return out


def fbp(plan: Plan, sino, window: str = "ram-lak", out_dtype=None):
    """Filtered back projection (2D fan beam) / FDK (3D circular cone beam) with a recon-mode
    plan: ramp filter into an FP32 buffer, then the recon-mode back projection."""
    import torch
    if plan.mode != "recon":
        raise ValueError("fbp needs a plan created with mode='recon'")
    q = torch.empty(sino.shape, dtype=torch.float32, device=sino.device)
    ctp_ramp_filter(plan, sino, q, window)
    return backproject(plan, q, out_dtype=out_dtype or torch.float32)


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


# ---- serving engine (include/ctserve.h) ------------------------------------------------------


def _torch_dtype(code: int):
    import torch
    return {CTP_F32: torch.float32, CTP_BF16: torch.bfloat16, CTP_F16: torch.float16}[code]


class Server:
    """Owner of a ``ctp_server*`` and of the device arena it sub-allocates (its HBM budget).

    ``submit`` queues a request and returns its ticket; ``wait`` returns the output as a tensor
    view into the arena (valid until ``release``).  The input tensor is kept referenced until its
    request has finished.  Outputs hold arena memory until released: a client that keeps every
    result can make later requests wait for memory that never frees (``wait`` then times out);
    admission needs one contiguous block per call.  Requests that have waited ``age_cap_s`` are
    served in arrival order; younger ones smallest first (``age_cap_s=0``: strict arrival
    order).  With ``express_work`` > 0 the last slot runs only requests of at most that many
    voxel-view updates, and longer requests run one at a time.  With ``launch_work`` > 0 each
    call is split into kernel launches of at most that many voxel-view updates (same results).
    """

    def __init__(self, arena_bytes: int, n_slots: int = 4, max_batch: int = 16, device=None,
                 age_cap_s: float = 0.05, express_work: float = 0.0, launch_work: float = 0.0):
        import torch
        self.device = torch.device(device or "cuda")
        # uint8 arena; torch's allocations are at least 256-byte aligned
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        cfg = _ServerConfig(self.arena.data_ptr(), int(arena_bytes), int(n_slots), int(max_batch),
                            int(round(age_cap_s * 1e6)), float(express_work),
                            float(launch_work))
        out = ctypes.c_void_p()
        _check(lib().ctp_server_create(ctypes.byref(cfg), ctypes.byref(out)), "ctp_server_create")
        self.handle = out
        self._pending = {}     # ticket -> (input tensor, plan, out dtype code, out shape)

    def submit(self, plan: Plan, direction: str, x, out_dtype=None, stream=None) -> int:
        """Queue ``A x`` (direction 'forward', x one volume) or ``A^T x`` ('backward', x one
        sinogram).  x must be a contiguous device tensor of one item."""
        g = plan.geom
        fwd = direction == "forward"
        if not fwd and direction != "backward":
            raise ValueError("direction must be 'forward' or 'backward'")
        shape_in = g.vol_shape if fwd else g.sino_shape
        _check_tensor(x, shape_in, "input")
        if x.numel() != int(np.prod(shape_in)):
            raise ValueError("a request holds exactly one item")
        in_code = _dtype_code(x)
        out_code = in_code if out_dtype is None else _dtype_code_of(out_dtype)
        t = ctypes.c_uint64()
        _check(lib().ctp_server_submit(self.handle, plan.handle, CTP_FORWARD if fwd else CTP_BACKWARD,
                                       x.data_ptr(), in_code, out_code, _stream_handle(stream),
                                       ctypes.byref(t)), "ctp_server_submit")
        self._pending[t.value] = (x, plan, out_code, tuple(g.sino_shape if fwd else g.vol_shape))
        return t.value

    def wait(self, ticket: int, timeout_s: Optional[float] = None):
        """Block until the request is done; its output as a view into the arena."""
        ptr = ctypes.c_void_p()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        _check(lib().ctp_server_wait(self.handle, ticket, us, ctypes.byref(ptr)), "ctp_server_wait")
        x, plan, out_code, shape = self._pending[ticket]
        self._pending[ticket] = (None, plan, out_code, shape)   # input no longer needed
        dt = _torch_dtype(out_code)
        off = ptr.value - self.arena.data_ptr()
        n = int(np.prod(shape)) * (4 if out_code == CTP_F32 else 2)
        return self.arena[off:off + n].view(dt).view(shape)

    def query(self, ticket: int) -> bool:
        done = ctypes.c_int()
        _check(lib().ctp_server_query(self.handle, ticket, ctypes.byref(done), None),
               "ctp_server_query")
        return bool(done.value)

    def info(self, ticket: int) -> dict:
        i = _RequestInfo()
        _check(lib().ctp_server_info(self.handle, ticket, ctypes.byref(i)), "ctp_server_info")
        return {"submit_ns": i.submit_ns, "admit_ns": i.admit_ns, "done_ns": i.done_ns,
                "batch": i.batch, "slot": i.slot}

    def cancel(self, ticket: int):
        """Remove a request that has not started; its wait then raises CtpError with status
        CTP_ECANCELED.  The ticket must still be released."""
        _check(lib().ctp_server_cancel(self.handle, ticket), "ctp_server_cancel")
        x, plan, out_code, shape = self._pending[ticket]
        self._pending[ticket] = (None, plan, out_code, shape)

    def release(self, ticket: int, stream=None):
        """Return the request's output to the arena once the work queued so far on ``stream``
        (default: the current stream) has run."""
        _check(lib().ctp_server_release(self.handle, ticket, _stream_handle(stream)),
               "ctp_server_release")
        self._pending.pop(ticket, None)

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().ctp_server_get_stats(self.handle, ctypes.byref(st)), "ctp_server_get_stats")
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if self.handle:
            h, self.handle = self.handle, ctypes.c_void_p()
            _check(lib().ctp_server_destroy(h), "ctp_server_destroy")
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def _dtype_code_of(dtype) -> int:
    import torch
    codes = {torch.float32: CTP_F32, torch.bfloat16: CTP_BF16, torch.float16: CTP_F16}
    if dtype not in codes:
        raise TypeError(f"unsupported dtype {dtype}: use float32, bfloat16 or float16")
    return codes[dtype]
