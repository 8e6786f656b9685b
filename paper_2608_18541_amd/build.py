"""Builds the gfx950 shared library ``libspinlattice.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
# translation units, compiled in parallel: the C ABI and one engine per precision
SOURCES = [os.path.join(PKG, "csrc", f)
           for f in ("spinlattice.hip", "sl_engine_fp32.hip", "sl_engine_fp64.hip")]
DEPS = [os.path.join(PKG, "csrc", f) for f in ("sl_device.hpp", "sl_kernels.hpp", "sl_engine.hpp")] + [
    os.path.join(os.path.dirname(PKG), "include", "spinlattice.h")]
LIB = os.path.join(PKG, "libspinlattice.so")
ARCH = os.environ.get("PYTORCH_ROCM_ARCH", "gfx950")


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def compile_flags() -> list:
    return ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
            # packed FP32 instructions stay off
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # multiply-adds are fused only within one source expression, so a
            # device function inlined into different kernels rounds the same
            "-ffp-contract=on",
            "-Wno-unused-command-line-argument"]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compiles the library (always when force) and returns its path: each
    translation unit to an object in parallel, then one shared link."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in SOURCES + DEPS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tag = "%d" % os.getpid()
    objs = [os.path.join(PKG, os.path.basename(src) + ".%s.o" % tag) for src in SOURCES]
    procs = [subprocess.Popen([hipcc()] + compile_flags() + ["-c", src, "-o", obj],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for src, obj in zip(SOURCES, objs)]
    errs = []
    for pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            errs.append(err[-4000:])
        elif verbose and err:
            print(err)
    try:
        if errs:
            raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
        tmp = LIB + ".tmp" + tag
        res = subprocess.run([hipcc(), "--offload-arch=" + ARCH, "-fPIC", "-shared"] + objs +
                             ["-o", tmp], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + res.stderr[-4000:])
        os.replace(tmp, LIB)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
