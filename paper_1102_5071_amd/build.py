"""Build libcfet.so (HIP for gfx950) in-tree with hipcc.

Usage:  python -m paper_1102_5071_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcfet.so")

SOURCES = ["device.hip", "persistent.hip", "sell.hip", "tile.hip", "batch.hip", "grad.hip", "api.cpp", "schemes.cpp",
           "host_common.cpp", "batch_api.cpp", "noalloc.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    "-fvisibility=hidden",
    # never emit packed FP32 instructions (see design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def source_digest() -> str:
    """SHA-256 over the library sources, the public header and the compiler
    flags: a counter measurement taken on one build is valid for another
    build only if the digests match."""
    import hashlib
    h = hashlib.sha256()
    h.update(" ".join(FLAGS).encode())
    files = sorted(os.listdir(CSRC)) + ["../../include/cfet.h"]
    for name in files:
        path = os.path.normpath(os.path.join(CSRC, name))
        if os.path.isfile(path) and not name.endswith((".so", ".o")):
            h.update(name.encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), *srcs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
