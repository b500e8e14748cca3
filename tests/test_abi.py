"""The C-ABI library: it builds, loads, exports every function include/ctproj.h declares,
and rejects bad descriptors before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2503_16741_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctproj.h")


@pytest.fixture(scope="module")
def ct():
    from paper_2503_16741_amd import ctproj, build
    if not os.path.exists(ctproj.LIB_PATH):
        build.build()
    ctproj.lib()
    return ctproj


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctp_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function(ct):
    names = declared_functions()
    assert len(names) == 10
    assert set(names) == set(ct.EXPORTED)
    lib = ct.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_server_header_exports(ct):
    text = open(os.path.join(ROOT, "include", "ctserve.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(ctp_[a-z_]+)\s*\(", text)))
    assert set(names) == set(ct.EXPORTED_SERVER)
    for n in names:
        assert hasattr(ct.lib(), n), n


def test_status_strings(ct):
    assert ct.ctp_status_string(0) == "ok"
    assert ct.ctp_status_string(-1) == "invalid argument"
    assert ct.ctp_status_string(-2) == "unsupported"
    assert ct.ctp_status_string(-3) == "out of memory"
    assert ct.ctp_status_string(-4) == "device error"
    assert ct.ctp_status_string(-5) == "timed out"


def test_server_argument_validation(ct):
    """Server entry points reject bad arguments before touching a device."""
    L = ct.lib()
    out = ctypes.c_void_p()
    assert L.ctp_server_create(None, ctypes.byref(out)) == -1
    bad = [(None, 1 << 20, 2, 4), (0x10000, 100, 2, 4), (0x10010, 1 << 20, 2, 4),
           (0x10000, 1 << 20, 0, 4), (0x10000, 1 << 20, 17, 4), (0x10000, 1 << 20, 2, 0),
           (0x10000, 1 << 20, 2, 1025)]
    for arena, nbytes, slots, mb in bad:
        cfg = ct._ServerConfig(arena, nbytes, slots, mb)
        assert L.ctp_server_create(ctypes.byref(cfg), ctypes.byref(out)) == -1, (arena, nbytes,
                                                                                 slots, mb)
    t = ctypes.c_uint64()
    assert L.ctp_server_submit(None, None, 0, None, 0, 0, None, ctypes.byref(t)) == -1
    assert L.ctp_server_wait(None, 1, 0, None) == -1
    done = ctypes.c_int()
    assert L.ctp_server_query(None, 1, ctypes.byref(done), None) == -1
    assert L.ctp_server_info(None, 1, None) == -1
    assert L.ctp_server_release(None, 1, None) == -1
    assert L.ctp_server_get_stats(None, None) == -1
    assert L.ctp_server_destroy(None) == 0


def geom(**over):
    kw = dict(kind="cone", det="flat", nx=8, ny=8, nz=8, dx=1.0, dy=1.0, dz=1.0, nu=16, nv=12,
              du=1.0, dv=1.0, n_views=4, theta=synth.full_circle(4), sad=100.0, sdd=200.0)
    kw.update(over)
    return synth.Geometry(**kw)


@pytest.mark.parametrize("over,method,status", [
    (dict(nx=0), "sf", -1),
    (dict(dy=-1.0), "sf", -1),
    (dict(sad=4.0, sdd=8.0), "sf", -1),              # source inside the object
    (dict(kind="cone_noncirc", det="curved"), "sf", -2),
    (dict(kind="cone_noncirc"), "dd", -2),
    (dict(det="curved", x_src=1.0), "sf", -2),
    (dict(phi=0.1), "sf", -1),                        # tilt needs a non-circular scan
    (dict(theta=np.zeros(3)), "sf", -1),              # vector length != n_views
    (dict(kind="fan2d", nz=1, nv=1, theta=np.array([0.0, np.nan, 1.0, 2.0])), "sf", -1),
    (dict(dx=1.0, du=0.01), "sf", -2),                # footprint wider than 16 columns
])
def test_plan_validation_without_device(ct, over, method, status):
    with pytest.raises(ct.CtpError) as e:
        ct.ctp_plan_create(geom(**over), method)
    assert e.value.status == status
    assert ct.ctp_last_error() != ""


@pytest.mark.parametrize("over,method,status", [
    (dict(), "dd", -2),                               # recon mode is SF only
    (dict(kind="cone_noncirc"), "sf", -2),            # and circular scans only
])
def test_recon_mode_validation_without_device(ct, over, method, status):
    with pytest.raises(ct.CtpError) as e:
        ct.ctp_plan_create(geom(**over), method, "recon")
    assert e.value.status == status
    L = ct.lib()
    d, keep = ct.make_desc(geom())
    out = ctypes.c_void_p()
    assert L.ctp_plan_create(ctypes.byref(d), 0, 7, ctypes.byref(out)) == ct.CTP_EINVAL
    assert L.ctp_ramp_filter(None, None, 0, None, 0, 1, 0, None) == ct.CTP_EINVAL


def test_null_arguments(ct):
    lib = ct.lib()
    out = ctypes.c_void_p()
    assert lib.ctp_plan_create(None, 0, 0, ctypes.byref(out)) == ct.CTP_EINVAL
    assert lib.ctp_plan_destroy(None) == ct.CTP_OK
    assert lib.ctp_project(None, None, 0, None, 0, 1, 0, None, 0, None) == ct.CTP_EINVAL
    assert lib.ctp_backproject(None, None, 0, None, 0, 1, 0, None, 0, None) == ct.CTP_EINVAL
    n = ctypes.c_size_t()
    assert lib.ctp_workspace_bytes(None, 0, 0, 0, 1, ctypes.byref(n)) == ct.CTP_EINVAL


def test_projector_module_arguments():
    """Projector(geom, mode, method, direction) validates its strings without a device."""
    from paper_2503_16741_amd.autograd import Projector
    g = geom()
    with pytest.raises(ValueError):
        Projector(g, "fbp", "SF", "forward")
    with pytest.raises(NotImplementedError):
        Projector(g, "proj", "VD", "forward")
    assert Projector(g, "recon", "SF", "backward").mode == "recon"
    with pytest.raises(ValueError):
        Projector(g, "proj", "SF", "sideways")
    p = Projector(g, "proj", "dd", "backward")
    assert p.method == "dd" and p.direction == "backward"


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with a message before touching a device."""
    import subprocess
    import sys
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
