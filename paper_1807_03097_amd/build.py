"""Build the igaefie HIP library (gfx950) in-tree: paper_1807_03097_amd/libigaefie.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libigaefie.so")
SOURCES = ["setup.cpp", "api.cpp", "kernels.hip", "kernels_batched.hip", "coupling.hip", "coupling_mfma.hip", "krylov.hip", "near_bf16.hip", "near_once.hip", "probe.hip", "serve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-fopenmp",
    # no packed-FP32 instruction selection
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


# host-code sanitizer variants (the device code is compiled as usual): used by the CPU
# tests of the host planning, never loaded by the GPU path
SANITIZE = {
    "asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"],
    "tsan": ["-Xarch_host", "-fsanitize=thread", "-Xarch_host", "-fno-omit-frame-pointer"],
}


def _newest_input(src: str) -> float:
    """latest modification time of a source and of every header it may include"""
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    inc = os.path.join(os.path.dirname(HERE), "include")
    hdrs += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return max(os.path.getmtime(p) for p in [src, *hdrs, __file__])


def build(verbose: bool = False, variant: str | None = None, incremental: bool = False) -> str:
    """Compile the library; variant "asan" or "tsan" builds a host-sanitized copy
    _build_<variant>/libigaefie_<variant>.so instead of libigaefie.so.  incremental:
    keep object files newer than their source, every header and this script."""
    extra = SANITIZE[variant] if variant else []
    objdir = os.path.join(HERE, "_build" + (f"_{variant}" if variant else ""))
    target = os.path.join(objdir, f"libigaefie_{variant}.so") if variant else OUT
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        spath = os.path.join(CSRC, src)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _newest_input(spath):
            continue
        cmd = [HIPCC, "-x", "hip", *FLAGS, *extra, "-c", spath, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if out.strip():
            sys.stderr.write(out)
        if p.returncode != 0:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = target + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fopenmp", *extra, "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose=True))
