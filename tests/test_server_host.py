"""The request server's scheduler on the CPU, under sanitizers.

tests/host/server_mock.cpp compiles csrc/server.hpp (admission, setup
workers, driver, polling, statistics), csrc/gate.hpp and the host plan code
against a stand-in handle whose setup and CG chunks take random host time.
Fed the geometries of 48 requests of the serving stream, every request must
come back with the outputs of its own ticket (or its injected failure), the
slot and memory caps must hold, and destroying the server with requests in
flight must leave no handle behind.  AddressSanitizer/UBSan (g++) and
ThreadSanitizer (ROCm's clang, whose runtime intercepts the condition
variable waits libstdc++ uses) must stay silent.
"""
import math
import os
import shutil
import subprocess
import sys

import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "server_mock.cpp")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def geometry(tmp_path_factory):
    path = tmp_path_factory.mktemp("srv") / "geom.txt"
    with open(path, "w") as f:
        for k in range(48):
            pr = W.serving_request(k)
            n = list(pr.n) + [1] * (3 - pr.dim)
            nsub = [len(c) - 1 for c in pr.cuts] + [1] * (3 - pr.dim)
            tau = 0.0 if math.isinf(pr.tau) else pr.tau
            f.write(" ".join(map(str, [pr.dim] + n + [tau] + nsub + [int(v) for c in pr.cuts for v in c])) + "\n")
    return str(path)


def _build(tmp_path_factory, compiler, flags, name):
    exe = str(tmp_path_factory.mktemp("srvbin") / name)
    subprocess.run([compiler, "-std=c++17", "-O1", "-g", "-pthread"] + flags + ["-o", exe, SRC], check=True,
                   capture_output=True)
    return exe


@pytest.fixture(scope="module")
def asan(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    return _build(tmp_path_factory, gxx, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                          "-Wno-subobject-linkage"], "server_asan")


@pytest.fixture(scope="module")
def tsan(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("clang with ThreadSanitizer not available")
    return _build(tmp_path_factory, CLANG, ["-fsanitize=thread"], "server_tsan")


def _run(exe, geometry, *args):
    res = subprocess.run([exe, geometry] + [str(a) for a in args], capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert out.strip().splitlines()[-1].startswith("OK"), out[-2000:]
    return out


@pytest.mark.parametrize("cap", [0, 1.05], ids=["uncapped", "capped"])
@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_server_scheduler_under_sanitizers(request, geometry, kind, cap):
    exe = request.getfixturevalue(kind)
    _run(exe, geometry, 4, 2, cap, 1, 0)          # serve all, check every ticket
    _run(exe, geometry, 3, 1, cap, 2, 1)          # destroy with the queue full
    _run(exe, geometry, 3, 2, cap, 3, 2)          # keyed problems: resident, solved in blocks


def _build_lib(tmp_path_factory, flags, name):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("srvlib") / name)
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-pthread", "-shared", "-fPIC", "-DSERVER_MOCK_LIB",
                    "-Wno-subobject-linkage"] + flags + ["-o", out, SRC], check=True, capture_output=True)
    return out


@pytest.mark.parametrize("kind", ["plain", "asan"])
def test_server_with_python_allocator_callbacks(tmp_path_factory, kind):
    """The device-memory hook set to Python callbacks (as a framework's caching
    allocator is): setup workers and the driver thread allocate and free
    through ctypes from native threads, with allocations refused now and then
    and servers destroyed with requests in flight.  Every request must return
    its own outputs or an out-of-memory error, every block must be handed
    back, and AddressSanitizer (preloaded into the Python process together with
    the C++ runtime it intercepts) must stay silent."""
    env = dict(os.environ)
    if kind == "asan":
        lib = _build_lib(tmp_path_factory, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"], "m_asan.so")
        gxx = shutil.which("g++")
        pre = [subprocess.run([gxx, f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
               for n in ("libasan.so", "libstdc++.so")]
        env["LD_PRELOAD"] = " ".join(pre)
        env["ASAN_OPTIONS"] = "detect_leaks=0"
    else:
        lib = _build_lib(tmp_path_factory, [], "m.so")
    driver = os.path.join(HERE, "host", "server_callbacks_driver.py")
    for fail_every in (0, 5):
        res = subprocess.run([sys.executable, driver, lib, "3", str(fail_every)], capture_output=True, text=True,
                             timeout=600, env=env)
        out = res.stdout + res.stderr
        assert res.returncode == 0, out[-4000:]
        assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
        assert out.strip().splitlines()[-1].startswith("OK"), out[-2000:]
