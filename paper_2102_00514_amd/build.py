"""Builds ``libsmoother.so`` (HIP, gfx950) next to this file.

    python -m paper_2102_00514_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
UNITS = ["smoother.hip", "engine_ct_f64.hip", "engine_ct_f32.hip", "engine_linear_f64.hip",
         "engine_linear_f32.hip", "engine_dense_ct_f64.hip", "engine_dense_ct_f32.hip", "warmstart.hip"]
LIB = os.path.join(PKG, "libsmoother.so")
# measurement kernels of the nx = 20 engine's matrix products (not linked into LIB)
PROBE_UNIT = "dense_probe.hip"
PROBE_LIB = os.path.join(PKG, "libdense_probe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".hip", ".hpp"))] + \
        [os.path.join(ROOT, "include", "smoother.h"), os.path.join(ROOT, "include", "warmstart.h")]


def build(verbose: bool = False, extra=(), jobs: int = 8) -> str:
    """Compiles every translation unit in parallel, then links the shared library."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    for unit in UNITS:
        obj = os.path.join(objdir, unit.replace(".hip", ".o"))
        cmd = [HIPCC, *HIP_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c", "-o", obj,
               os.path.join(CSRC, unit)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((unit, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                  text=True)))
        while sum(p.poll() is None for _, _, p in procs) >= jobs:
            time.sleep(0.2)
    failed = []
    for unit, obj, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed.append(unit)
    if failed:
        raise RuntimeError(f"hipcc failed on {failed}")
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in procs]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libsmoother.so failed")
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """libdense_probe.so: the FP64 VALU and MFMA forms of the nx = 20 products."""
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC, *HIP_FLAGS, "-shared", "-I", os.path.join(ROOT, "include"), "-o", tmp,
           os.path.join(CSRC, PROBE_UNIT)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("building libdense_probe.so failed")
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    if not os.path.exists(PROBE_LIB) or os.path.getmtime(PROBE_LIB) < t:
        return True
    return any(os.path.getmtime(s) > t for s in sources())


if __name__ == "__main__":
    print(build(verbose=True))
