"""Build the HIP library (gfx950) in-tree: paper_2110_03636_amd/libhkkt.so."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhkkt.so")
SOURCES = [os.path.join(CSRC, "hkkt.hip"), os.path.join(CSRC, "analysis.cpp")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("analysis.hpp", "kernels.hpp", "kernels.inl")] + [
    os.path.join(os.path.dirname(HERE), "include", "hkkt.h")]


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags(debug: bool = False):
    f = ["--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Wno-unused-result",
         # packed FP32 VALU forms are avoided on this target
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    f += ["-O0", "-g"] if debug else ["-O3"]
    return f


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(d) <= t for d in DEPS):
            return LIB
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + flags() + ["-o", tmp] + SOURCES
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-8000:])
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
