"""Compile libgw.so (HIP kernels + C ABI + host grids) for gfx950, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgw.so")
SOURCES = ["gw_kernels.hip", "gw_api.hip", "grids.cpp", "ir.cpp"]


def source_hash():
    """sha256 of the kernel and ABI sources (names counter summaries to a build)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gw_kernels.hip", "gw_kernels.h", "gw_api.hip"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hipcc():
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if p and os.path.exists(p):
            return p
    raise RuntimeError("hipcc not found")


def build(verbose=False, arch="gfx950"):
    out_tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # MFMA accumulators in arch VGPRs: avoids per-iteration AGPR copies
           "-mllvm", "-amdgpu-mfma-vgpr-form",
           "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include"),
           "-o", out_tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msg)
    if verbose and msg.strip():
        print(msg, file=sys.stderr)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
