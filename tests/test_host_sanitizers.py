"""The library's host code (geometry validation, unknowns, cluster and block-cluster
trees, near-field layouts, error handling) under AddressSanitizer + UndefinedBehavior-
Sanitizer and under ThreadSanitizer: the library is rebuilt with host-side sanitizers
(paper_1807_03097_amd/build.py, variants asan and tsan; device code unchanged) and
tests/host_driver.cpp plans operators on one thread and on eight threads at once (one
host-only context per thread, one geometry shared by all).  No device calls."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1807_03097_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"   # the driver is plain C++ (no HIP)
DRIVER_FLAGS = {"asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                "tsan": ["-fsanitize=thread"]}

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)),
                                reason="hipcc / clang++ not available")


def _write_geom(path, patches):
    deg, nctrl, knots, ctrl = W.pack(patches)
    with open(path, "wb") as f:
        np.array([len(patches)], np.int32).tofile(f)
        deg.astype(np.int32).tofile(f)
        nctrl.astype(np.int32).tofile(f)
        np.array([len(knots)], np.int64).tofile(f)
        knots.astype(np.float64).tofile(f)
        np.array([len(ctrl)], np.int64).tofile(f)
        ctrl.astype(np.float64).tofile(f)


@pytest.mark.slow
@pytest.mark.parametrize("variant", ["asan", "tsan"])
def test_host_code_under_sanitizers(tmp_path, variant):
    from paper_1807_03097_amd import build as B
    lib = B.build(variant=variant, incremental=True)   # objects older than their inputs are rebuilt
    libdir = os.path.dirname(lib)
    exe = str(tmp_path / f"host_driver_{variant}")
    cmd = [CLANGXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *DRIVER_FLAGS[variant], "-o", exe,
           os.path.join(ROOT, "tests", "host_driver.cpp"), f"-L{libdir}", f"-l:libigaefie_{variant}.so",
           f"-Wl,-rpath,{libdir}", "-lpthread"]
    cp = subprocess.run(cmd, capture_output=True, text=True)
    assert cp.returncode == 0, cp.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    for name, pats in (("sphere", W.cube_sphere()), ("torus", W.torus())):
        gpath = str(tmp_path / f"{name}.geom")
        _write_geom(gpath, pats)
        r = subprocess.run([exe, gpath, "8"], env=env, capture_output=True, text=True, timeout=600)
        out = r.stdout + r.stderr
        print(out[-3000:])
        assert r.returncode == 0, out[-3000:]
        assert "all checks passed" in out
        for bad in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer", "ERROR: LeakSanitizer"):
            assert bad not in out
