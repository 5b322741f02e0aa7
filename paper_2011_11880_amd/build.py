"""Build libpf.so (host setup + C ABI with g++, device code with hipcc for gfx950).

Usage: python -m paper_2011_11880_amd.build   (or call build()).
The library lands next to this file so that it ships with the source tree.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpf.so")
BUILD_DIR = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HOST_SRCS = ["pf_setup.cpp", "pf_api.cpp"]
DEVICE_SRCS = ["pf_device.hip", "pf_lu.hip", "pf_qlim.hip", "pf_batchlu.hip"]

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # every floating-point contraction in the kernels is written out with fma()
    "-ffp-contract=off",
    # no packed FP32 instructions on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False) -> str:
    """Compile every source and link libpf.so; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    inc = ["-I", INCLUDE, "-I", CSRC]
    for s in HOST_SRCS:
        o = os.path.join(BUILD_DIR, s + ".o")
        _run(["g++", *HOST_FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    # the tune cache keys schedules by the kernel source they were timed on
    tag = [f'-DPF_KERNEL_SHA="{kernel_source_hash()}"']
    for s in DEVICE_SRCS:
        o = os.path.join(BUILD_DIR, s + ".o")
        out = _run([HIPCC, *HIP_FLAGS, *tag, *inc, "-c", os.path.join(CSRC, s), "-o", o])
        if verbose and out.strip():
            print(out)
        objs.append(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-ldl", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


# Where the kernel-relevant text of each hashed source ends: the host-side
# drivers at the end of pf_device.hip, and the host plan and declarations of
# pf_internal.hpp (the constants and the grid record before it are read by
# the kernels).
_HASH_CUTS = (("pf_device.hip", "// Host-side drivers:"),
              ("pf_internal.hpp", "struct HostPlan {"))


def kernel_source_hash() -> str:
    """Short hash of the evaluation and adjoint kernels' source and their
    launch code (ties tune-cache entries and counter summaries to the kernel
    they were taken on).  Host-only code below the cut lines is left out, so
    changing it keeps cached schedules and summaries valid."""
    import hashlib
    h = hashlib.sha256()
    for f, cut in _HASH_CUTS:
        with open(os.path.join(CSRC, f), "rb") as fh:
            text = fh.read()
        at = text.find(cut.encode())
        if at < 0:
            raise RuntimeError(f"{f}: cut line {cut!r} not found")
        h.update(text[:at])
    return h.hexdigest()[:16]


def clean():
    shutil.rmtree(BUILD_DIR, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose=True))
