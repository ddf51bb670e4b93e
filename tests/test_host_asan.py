"""Host AddressSanitizer run of the library's planning and validation code.

The C-ABI sources that hold the planning (api.cpp, timing.cpp) are compiled
with AddressSanitizer on their host side and linked with the kernel objects
and the driver in tests/host_asan/driver.cpp. The driver calls only entry
points that return before any HIP call: workspace queries over random shapes,
argument rejection on every entry point, and batch planning into host memory.
Runs on the CPU (no device is touched).
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_04840_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
DRIVER = os.path.join(ROOT, "tests", "host_asan", "driver.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["--offload-arch=gfx950", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result", "-Wno-unused-value"]
ASAN = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])
    return r


def _kernel_object(name: str, tmp: str) -> str:
    """The package build's object for a kernel source when it is newer than
    its sources, else a fresh compile (the kernels are not instrumented)."""
    obj = os.path.join(BUILD, name + ".o")
    deps = [os.path.join(CSRC, f) for f in (name + ".hip", "common.hpp", "internal.hpp")] + [
        os.path.join(INCLUDE, "tucker.h")]
    if os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps):
        return obj
    out = os.path.join(tmp, name + ".o")
    _run([HIPCC] + COMMON + ["-O3", "-c", os.path.join(CSRC, name + ".hip"), "-o", out])
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_planning_and_validation_under_address_sanitizer(tmp_path):
    tmp = str(tmp_path)
    objs = []
    for src in ("api.cpp", "timing.cpp"):
        out = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
        _run([HIPCC, "-x", "hip"] + COMMON + ASAN + ["-c", os.path.join(CSRC, src), "-o", out])
        objs.append(out)
    drv = os.path.join(tmp, "driver.o")
    _run([HIPCC, "-x", "hip"] + COMMON + ASAN + ["-c", DRIVER, "-o", drv])
    objs += [drv, _kernel_object("ttm", tmp), _kernel_object("orth", tmp)]
    exe = os.path.join(tmp, "driver")
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address"] + objs + ["-o", exe])
    # the sanitizer runtime is linked in (a build without it would pass silently)
    nm = shutil.which("nm") or "/usr/bin/nm"
    assert "__asan_init" in _run([nm, exe]).stdout
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "all checks passed" in r.stdout, r.stdout[-2000:] + r.stderr[-6000:]
