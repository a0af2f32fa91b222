"""Build the HIP library (libcow.so) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcow.so")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # exact fp32 decision sequences: no contraction, IEEE divide/sqrt
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    # hardware fp32 atomics for the backward scatter
    "-munsafe-fp-atomics",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
]


SOURCES = ("cow_march.hip", "cow_march_bwd.hip", "cow_mlp.hip", "cow_reg.hip", "cow_gather.hip", "cow_host.cpp")


def source_digest():
    """First 16 hex digits of the SHA-256 of the library's sources and headers
    (part of the autotuner's cache key)."""
    h = hashlib.sha256()
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h")))
    for f in names:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    with open(os.path.join(ROOT, "include", "cow.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def build_library(verbose=False):
    srcs = [os.path.join(CSRC, f) for f in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + HIP_FLAGS + [f'-DCOW_SOURCE_DIGEST="{source_digest()}"', "-I", os.path.join(ROOT, "include"),
                                   "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd, stderr=None if verbose else subprocess.DEVNULL)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
