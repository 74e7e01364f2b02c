"""Build the gfx950 shared library ``libmgir.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmgir.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# FP contraction is off so that every kernel and launch shape forms the same
# roundings; packed FP32 instructions are disabled.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def _stale(obj, srcs):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(s) > t for s in srcs)


SOURCES = (("mg_kernels.hip", True), ("mg_multi.hip", True), ("mg_tail.hip", True), ("mg_sweep_update.hip", True),
           ("mg_smooth_restrict.hip", True),
           ("mg_rescale.hip", True),
           ("mg_cg.hip", True),
           ("mg_q1.hip", True),
           ("mg_noalloc.hip", True),
           ("mg_api.cpp", False))


def build(force: bool = True) -> str:
    """Compile (all sources in parallel) and link; with force=False only
    objects older than a source or header are rebuilt."""
    os.makedirs(BUILD, exist_ok=True)
    objs, jobs = [], []
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers.append(os.path.join(ROOT, "include", "mgir.h"))
    for src, dev in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        if not force and not _stale(obj, [os.path.join(CSRC, src)] + headers):
            continue
        if dev:
            cmd = [HIPCC, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE
        else:
            cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c",
                   os.path.join(CSRC, src), "-o", obj] + COMMON
        print("+", " ".join(cmd), flush=True)
        jobs.append((src, subprocess.Popen(cmd)))
    failed = [src for src, p in jobs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc " + " ".join(failed))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv)
    sys.exit(0)
