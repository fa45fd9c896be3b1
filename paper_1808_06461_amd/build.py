"""Builds the in-tree HIP library libchn.so for gfx950 (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libchn.so")
HIP_SOURCES = ["api.hip", "plane.hip", "plane_zinv_f.hip", "plane_zinv_d.hip", "plane_xpass_f.hip",
               "plane_xpass_d.hip", "plane_zfwd_f.hip", "plane_zfwd_d.hip", "plane_batch.hip", "pencil.hip",
               "lowstorage.hip"]
HOST_SOURCES = ["coeffs.cpp", "meshopt.cpp"]
ARCH = os.environ.get("CHN_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
# -ffp-contract=on: products are fused into FMAs within a source expression
# only, never across statements, so a kernel body gives the same bits in every
# kernel that inlines it (an ensemble's batched launches and a single
# context's launches agree bit for bit)
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-ffp-contract=on"]


def _run(cmd):
    r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[-1]}")
    return r


def build(verbose=False):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []  # (command, object); compiled concurrently
    for src in HOST_SOURCES:  # plain host C++ (quad precision tables)
        o = os.path.join(objdir, src + ".o")
        jobs.append(([HIPCC, "-x", "c++", *COMMON, "-c", src, "-o", o], o))
    for src in HIP_SOURCES:
        o = os.path.join(objdir, src + ".o")
        jobs.append(([HIPCC, "-x", "hip", *COMMON, *DEVICE, "-c", src, "-o", o], o))
    procs = [(subprocess.Popen(cmd, cwd=CSRC, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True), cmd)
             for cmd, _ in jobs]
    failed = None
    for p, cmd in procs:
        out, err = p.communicate()
        if p.returncode != 0 and failed is None:
            sys.stderr.write(" ".join(cmd) + "\n" + out + err)
            failed = cmd[-1]
    if failed:
        raise RuntimeError(f"build step failed: {failed}")
    objs = [o for _, o in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
