"""Measurement of the nx = 20 engine's wave routines (libdense_probe.so, built
by paper_2102_00514_amd.build).

    python -m paper_2102_00514_amd.dense_probe [--blocks B] [--reps R]
    python -m paper_2102_00514_amd.dense_probe --phases [--blocks B] [--reps R]

The first form compares the 20 x 20 x 20 FP64 products, the VALU routine
against the engine's FP64 MFMA routine (v_mfma_f64_16x16x4f64), on the engine's
LDS layout: per variant the kernel time (HIP events, best of 5 launches) for B
blocks (one wavefront each) of R chained products, the time per product and per
wavefront, and the largest difference of the two results relative to the
result's scale.  The second prints the shader-clock cycles per call of each
routine an eq. 15 combine is made of, and of the whole combine, the carry
application and the eq. 19 combine, on one wavefront (B = 1) or on B at once.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
N = 20


def load():
    path = os.path.join(PKG, "libdense_probe.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2102_00514_amd.build")
    lib = ctypes.CDLL(path)
    lib.dprobe_products.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]
    lib.dprobe_products.restype = ctypes.c_int
    lib.dprobe_phase_count.argtypes = []
    lib.dprobe_phase_count.restype = ctypes.c_int
    lib.dprobe_phases.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.dprobe_phases.restype = ctypes.c_int
    return lib


PHASES = ("copy", "cholesky", "product", "product_At", "copy_transposed", "forward_substitution_20_rhs",
          "matrix_vector", "symmetrise", "filter_combine_eq15", "carry_application", "smoother_combine_eq19")


def phases(blocks: int = 1, reps: int = 20) -> dict:
    """Mean shader-clock cycles per call of each routine (over blocks and reps)."""
    import torch
    lib = load()
    assert lib.dprobe_phase_count() == len(PHASES)
    out = torch.zeros((blocks, len(PHASES)), dtype=torch.int64, device="cuda")
    st = lib.dprobe_phases(blocks, reps, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    if st != 0:
        raise RuntimeError(f"dprobe_phases failed with hipError {st}")
    torch.cuda.synchronize()
    mean = out.to(torch.float64).mean(dim=0) / reps
    return {name: round(float(v), 1) for name, v in zip(PHASES, mean)}


def products(lib, variant: int, A, B, reps: int, stream: int):
    """C = reps * A B per block on the device (A, B torch float64 [blocks, 20, 20])."""
    import torch
    C = torch.empty_like(A)
    st = lib.dprobe_products(variant, A.shape[0], reps, A.data_ptr(), B.data_ptr(), C.data_ptr(), stream)
    if st != 0:
        raise RuntimeError(f"dprobe_products failed with hipError {st}")
    return C


def measure(blocks: int = 2048, reps: int = 64, seed: int = 0) -> dict:
    import torch
    lib = load()
    g = torch.Generator().manual_seed(seed)
    A = torch.randn((blocks, N, N), generator=g, dtype=torch.float64).cuda()
    B = torch.randn((blocks, N, N), generator=g, dtype=torch.float64).cuda()
    stream = torch.cuda.current_stream()
    out = {"blocks": blocks, "reps": reps, "n": N}
    res = {}
    for name, v in (("valu", 0), ("mfma_f64", 1)):
        products(lib, v, A, B, reps, stream.cuda_stream)      # warm-up
        best = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            C = products(lib, v, A, B, reps, stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None or ms < best else best
        res[name] = C
        out[name] = {"kernel_ms": round(best, 4),
                     "ns_per_product": round(best * 1e6 / (blocks * reps), 3),
                     "useful_gflops": round(2 * N ** 3 * blocks * reps / (best * 1e-3) / 1e9, 2)}
    scale = float(res["valu"].abs().max())
    out["max_rel_diff"] = float((res["valu"] - res["mfma_f64"]).abs().max()) / scale
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--blocks", type=int, default=None)
    ap.add_argument("--reps", type=int, default=None)
    ap.add_argument("--phases", action="store_true", help="cycles per call of the wave routines")
    args = ap.parse_args(argv)
    if args.phases:
        blocks = args.blocks or 1
        print(json.dumps({"blocks": blocks, "cycles_per_call": phases(blocks, args.reps or 20)}), flush=True)
        return
    r = measure(args.blocks or 2048, args.reps or 64)
    lat = measure(1, args.reps or 64, seed=1)
    r["single_wavefront"] = {k: lat[k] for k in ("valu", "mfma_f64")}
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
