"""Build the HIP engine (libvp.so) for gfx950 with hipcc, in-tree.

-ffp-contract=off keeps every multiply and add a separate rounding (fma only
where the source writes it); packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "vp_engine.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "vp_kernels.hpp"),
        os.path.join(ROOT, "include", "vp.h")]
LIB = os.path.join(HERE, "libvp.so")
SRC4 = os.path.join(HERE, "csrc", "vp4_engine.hip")
LIB4 = os.path.join(HERE, "libvp4.so")
ARCH = os.environ.get("VP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
              shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include")]


def _compile(src: str, out: str, verbose: bool, extra=()) -> str:
    tmp = out + ".tmp"
    cmd = [hipcc()] + flags() + list(extra) + ["-o", tmp, src]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"{os.path.basename(out)} build failed:\n" +
                           res.stderr[-6000:])
    if verbose:
        print(" ".join(cmd))
        if res.stderr:
            print(res.stderr[-3000:])
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, out: str = LIB, extra=()) -> str:
    """Compile libvp.so (the 2D phase-space engine) and libvp4.so (the 4D
    one); always rebuilds, atomic replace of the outputs."""
    _compile(SRC4, LIB4, verbose, extra)
    return _compile(SRC, out, verbose, extra)


if __name__ == "__main__":
    print(build(verbose=True))
