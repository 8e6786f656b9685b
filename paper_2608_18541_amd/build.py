"""Builds the gfx950 shared library ``libspinlattice.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(PKG, "csrc", "spinlattice.hip")
DEPS = [os.path.join(PKG, "csrc", f) for f in ("sl_device.hpp", "sl_kernels.hpp")] + [
    os.path.join(os.path.dirname(PKG), "include", "spinlattice.h")]
LIB = os.path.join(PKG, "libspinlattice.so")
ARCH = os.environ.get("PYTORCH_ROCM_ARCH", "gfx950")


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def compile_flags() -> list:
    return ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-shared",
            # packed FP32 instructions stay off
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # multiply-adds are fused only within one source expression, so a
            # device function inlined into different kernels rounds the same
            "-ffp-contract=on",
            "-Wno-unused-command-line-argument"]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compiles the library (always when force) and returns its path."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in [SRC] + DEPS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + compile_flags() + [SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-4000:])
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
