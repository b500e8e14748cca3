"""Host-side pieces that need no GPU: the serving engine's arena allocator and batch choice
(compiled with g++ and sanitizers against csrc/serve_host.h), and the C structs of the public
headers against the ctypes mirrors used by the Python binding."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _cc(tmp_path, src, out, lang_flags, extra=()):
    exe = str(tmp_path / out)
    cmd = list(lang_flags) + ["-o", exe, src] + list(extra)
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=180)
    assert res.returncode == 0, res.stdout + res.stderr
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_serve_host_allocator_and_batching(tmp_path):
    exe = _cc(tmp_path, os.path.join(ROOT, "tests", "host", "serve_host_test.cpp"), "sht",
              ["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout + res.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_serving_engine_simulated_device(tmp_path):
    """csrc/server.cpp compiled unchanged against a simulated device (streams with timed work,
    events, stub projector calls with the library's workspace formulas): bursts of mixed
    requests whose outputs the client holds until all are done must all complete, with every
    call given a large enough workspace.  A scratch block placed between outputs used to leave
    a request that could never be admitted (fragmentation); scratch now comes from the top.
    Failure injection: calls that fail to launch or fail on the device fail only their own
    requests, the others complete and the arena empties; queued requests can be cancelled;
    short requests overtake long ones until the age cap, then arrival order holds."""
    exe = _cc(tmp_path, os.path.join(ROOT, "tests", "host", "serve_sim.cpp"), "sim",
              ["g++", "-std=c++17", "-O1", "-pthread", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "tests", "host", "fakehip")])
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout + res.stderr


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "ctserve.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
#define S(T) printf(#T " %zu\n", sizeof(T))
int main(void) {
    S(ctp_geometry_desc); P(ctp_geometry_desc, dx); P(ctp_geometry_desc, nu);
    P(ctp_geometry_desc, du); P(ctp_geometry_desc, n_views); P(ctp_geometry_desc, theta);
    P(ctp_geometry_desc, v_ofst); P(ctp_geometry_desc, len_theta); P(ctp_geometry_desc, len_v_ofst);
    S(ctp_server_config); P(ctp_server_config, arena_bytes); P(ctp_server_config, n_slots);
    P(ctp_server_config, max_batch); P(ctp_server_config, age_cap_us);
    P(ctp_server_config, express_work); P(ctp_server_config, launch_work);
    S(ctp_request_info); P(ctp_request_info, done_ns); P(ctp_request_info, batch);
    P(ctp_request_info, slot);
    S(ctp_server_stats); P(ctp_server_stats, calls); P(ctp_server_stats, cancelled);
    P(ctp_server_stats, max_running);
    P(ctp_server_stats, max_batch_seen); P(ctp_server_stats, arena_peak);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs gcc and the HIP headers")
def test_ctypes_structs_match_headers(tmp_path):
    from paper_2503_16741_amd import ctproj
    src = tmp_path / "probe.c"
    src.write_text(PROBE)
    exe = _cc(tmp_path, str(src), "probe",
              ["gcc", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
               "-I" + os.path.join(ROOT, "include")])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60).stdout
    c = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    mirrors = {"ctp_geometry_desc": ctproj._Desc, "ctp_server_config": ctproj._ServerConfig,
               "ctp_request_info": ctproj._RequestInfo, "ctp_server_stats": ctproj._ServerStats}
    for key, val in c.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(mirrors[t], f).offset == int(val), key
        else:
            assert ctypes.sizeof(mirrors[key]) == int(val), key
