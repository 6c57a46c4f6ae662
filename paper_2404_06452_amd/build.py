"""Builds libpaam.so (hipcc, gfx950) and the input generator (gcc), in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBPAAM = os.path.join(PKG, "libpaam.so")

SOURCES = ["paam_host.cpp", "paam_kernels.hip", "paam_surrogate.hip", "paam_units.hip", "paam_des.hip"]
HEADERS = [os.path.join(CSRC, h) for h in ("paam_internal.h", "paam_device.h")] + [
    os.path.join(INCLUDE, "paam.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def build_libpaam(force: bool = True) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    if not force and os.path.exists(LIBPAAM):
        newest = max(os.path.getmtime(p) for p in srcs + HEADERS)
        if os.path.getmtime(LIBPAAM) >= newest:
            return LIBPAAM
    tmp = LIBPAAM + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", INCLUDE, "-I", CSRC, "-o", tmp] + srcs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for libpaam")
    os.replace(tmp, LIBPAAM)
    return LIBPAAM


def build_all(force: bool = True) -> None:
    from . import chaingen
    chaingen.build(force=force)
    build_libpaam(force=force)


if __name__ == "__main__":
    build_all(force=True)
    print(LIBPAAM)
