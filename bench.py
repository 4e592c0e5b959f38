"""Benchmark: smoothed steps per second per iteration of the parallel iterated
smoother on one MI355X.

Workload (default): coordinated-turn target, two bearing sensors, T = 2^15
measurements (32769 slots), FP64, Taylor (IEKS) linearisation.  One "step" of
this benchmark is one full iteration of the method: linearise every slot,
build the filtering elements, prefix-scan them, build the smoothing elements,
suffix-scan them, and reduce the convergence statistic.  Inputs are resident
on the GPU before timing starts.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--lin taylor|cubature|unscented]
                    [--workload c2|c3|c5|c5batch|c2sweep]

Other workloads (one JSON line each): c3, 4096 ragged tracks with T_i ~ U{100..8192}
(cubature; steps = sum of T_i per iteration); c5, four stacked targets (nx = 20,
eight bearings, T = 2^16, unscented) on the wavefront-cooperative engine, whose
roofline is FP64 arithmetic; c5batch, 256 such tracks with T_i ~ U{1024..65536}
in one ragged batch (~8.5e6 slots, ~133 GB of device memory); c2sweep, T = 2^10..2^15 on the GPU parallel and
sequential paths (FP64 and FP32) and the CPU oracle.  The learned warm-start
comparison runs with c2.

Prints one JSON line on stdout; details go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "smoothed steps/sec per iteration at T=2^15 FP64; time-to-converge learned vs plain"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def scan_bytes_per_slot(n: int, word: int) -> dict:
    """Algorithmic bytes of the method per slot and iteration: each scan reads
    its materialised elements once and writes its outputs once.  Forward scan
    (eq. 15): filtering element (A, b, C, eta, J) in, filtered mean and packed
    covariance out; reverse scan (eq. 19): smoothing element (E, g, L) in,
    smoothed mean and packed covariance out."""
    s = n * (n + 1) // 2
    fwd = (n * n + 2 * n + 2 * s) + (n + s)
    rev = (n * n + n + s) + (n + s)
    return {"forward": fwd * word, "reverse": rev * word, "iteration": (fwd + rev) * word}


# Which scan each n = 5 kernel belongs to (its algorithmic bytes are that
# scan's per slot, or per tile aggregate for the top scans).  The separate
# sigma-point linearisation pass produces the elements' inputs and is not
# charged any of the scans' bytes.
KERNEL_SCAN = {"forward_up": "forward", "tiles_up_filter": "forward",
               "tiles_top_filter": "forward", "tiles_down_filter": "forward",
               "forward_down_backward_up": "reverse", "backward_down": "reverse",
               "tiles_up_smoother": "reverse", "tiles_top_smoother": "reverse", "tiles_down_smoother": "reverse",
               "sequential": "iteration"}


def design_bytes_per_position(kernel: str, n: int, p: int, lin: str, word: int, K: int) -> float:
    """Bytes each kernel of this design moves per slot when every input it
    reads is read once and every output it writes is written once, including
    the intermediates of the design (stored transitions, lane prefixes, stored
    elements for K > 1).  K = slots per lane, so lane-level scan state is
    amortised over K slots.  Reported beside the algorithmic bytes."""
    s = n * (n + 1) // 2
    sp = p * (p + 1) // 2
    fe = n * n + 2 * n + 2 * s          # filtering element (A, b, C, eta, J)
    se = n * n + n + s                  # smoothing element (E, g, L)
    car = n + s                         # trajectory slot (mean, packed covariance)
    tr = n * n + n + s                  # transition rows (F, c, Q') of the stored linearisation
    lin_words = n * n + n + s + p * n + p + sp + p
    xin = n + (s if lin != "taylor" else 0)   # linearisation point (mean [+ covariance])
    # Filtering elements are never stored: the forward down-sweep builds them
    # again (K > 1) from the linearisation point (Taylor) or the stored
    # linearisation (sigma points); Taylor transitions are evaluated again for
    # the smoothing elements.  With K = 1 the down-sweeps start from each
    # lane's inclusive prefix; smoothing elements are stored only for K > 1.
    ke = 1 if K > 1 else 0
    taylor = lin == "taylor"
    words = {
        # linearisation inputs + lane prefix
        "forward_up": (xin + p if taylor else lin_words) + fe / K,
        # linearisation inputs again + carries + smoothing element (K > 1) + reverse lane prefix
        "forward_down_backward_up": ((n + ke * p) if taylor else (lin_words if ke else tr)) + fe / K
                                    + ke * se + se / K,
        # reverse carries, new trajectory in place, convergence statistic (reads old means)
        "backward_down": ke * se + se / K + n + car,
        "tiles_up_filter": fe + fe / 2, "tiles_top_filter": fe + car, "tiles_down_filter": fe + fe / 2 + car,
        # (per tile aggregate: read once, write its carry)
        "tiles_up_smoother": se + se / 2, "tiles_top_smoother": se + car, "tiles_down_smoother": se + se / 2 + car,
        "linearize": xin + p + lin_words,
        "sequential": lin_words + 2 * car,
        "delta": 2 * n,
        "reset_delta": 1,
    }[kernel]
    return words * word


# Floating-point operations per position of the wavefront-cooperative (n = 20)
# kernels, counted from their dense 20 x 20 products (2 N^3 each), Cholesky
# factorisations (N^3 / 3), triangular solves with N right-hand sides (N^3) and
# the sigma-point statistics; vector and O(N^2) terms are left out.
def dense_flops_per_position(kernel: str, n: int, p: int) -> float:
    mm, ch, sv = 2 * n ** 3, n ** 3 / 3, n ** 3
    m = 2 * n + 1                                   # sigma points
    f_lin = ch + 2 * m * n * n + 2 * n ** 3 + sv    # Phi, D^T D, G
    h_lin = 2 * m * p * p + 2 * n * p * p + n * n * p
    element = 2 * (2 * p * n * n) + 2 * p * p * n + 3 * (2 * n * n * p) + 2 * p * p * n
    combine_f = 10 * mm + 2 * ch + sv
    apply_f = 5 * mm + 2 * ch + sv
    combine_s, apply_s = 3 * mm, 2 * mm
    smoother_element = 3 * mm + ch + 2 * sv
    return {
        "dn_linearize": f_lin + h_lin,
        "dn_forward_up": element + combine_f,
        "dn_forward_down_backward_up": apply_f + smoother_element + combine_s,
        "dn_backward_down": apply_s,
        "scan_up_filter": combine_f, "scan_down_filter": apply_f,
        "scan_up_smoother": combine_s, "scan_down_smoother": apply_s,
        "reset_delta": 0.0,
    }[kernel]


PROFILE_REPEAT = 8   # launches of a kernel between one pair of HIP events in the profiling pass

# Sources of the n = 5 kernels whose HBM traffic is recorded in profiles/
# (the kernels, their device functions and their launch configuration).
TRAFFIC_SOURCES = ("fused.hpp", "elements.hpp", "operators.hpp", "sqrt.hpp", "linalg.hpp", "models.hpp", "scan.hpp",
                   "slot_kernels.hpp", "engine.hpp", "engine_ct_f64.hip")


def kernel_sources_sha256() -> str:
    """Hash of the sources that define the n = 5 kernels and their launches."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2102_00514_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(TRAFFIC_SOURCES):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when there is none for this kernel/workload or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("csrc_sha256") != kernel_sources_sha256():
        return None
    return rec["bytes_per_launch"]


def host_cpu() -> dict:
    """CPU model string and logical CPU count of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


_NATIVE_ORACLE = None


def native_oracle():
    """The oracle compiled with -O3 -march=native for this host (built once per run)."""
    global _NATIVE_ORACLE
    import tempfile

    import oracle
    if _NATIVE_ORACLE is None:
        _NATIVE_ORACLE = oracle.build_native(tempfile.mkdtemp(prefix="oracle_native_"))
        oracle.use_library(_NATIVE_ORACLE)
    return oracle


def cpu_baseline(pb, lin: str, budget_s: float, threads: int = 1) -> dict:
    """The oracle, untuned (gcc -O3 -march=native), on a bounded sample of the
    same workload: one iteration from the prior broadcast per track, track
    after track (a single track repeats; a track longer than the budget allows
    is cut to a prefix), until about budget_s seconds have been spent.  With
    threads > 1 independent tracks run on that many host threads at once (the
    oracle call releases the interpreter lock)."""
    import threading

    oracle = native_oracle()
    first = pb.track(0)
    T0 = int(first.offsets[1])
    # one-iteration cost probe on a short prefix decides whether the full track fits
    probe_T = min(T0, 256)
    tp = time.perf_counter()
    oracle.smoother(first.prefix(probe_T) if probe_T < T0 else first, 1, lin, filtered=False)
    per_step = (time.perf_counter() - tp) / probe_T
    cut = T0 if per_step * T0 <= budget_s else max(probe_T, int(budget_s / 3 / per_step))
    lock = threading.Lock()
    state = {"next": 0, "steps": 0, "iters": 0}
    t0 = time.perf_counter()

    def worker():
        while True:
            with lock:
                if time.perf_counter() - t0 >= budget_s:
                    return
                i = state["next"]
                state["next"] += 1
            tr = pb.track(i % pb.n_tracks)
            T = int(tr.offsets[1])
            if T > cut:
                tr, T = tr.prefix(cut), cut
            oracle.smoother(tr, 1, lin, filtered=False)
            with lock:
                state["steps"] += T
                state["iters"] += 1

    pool = [threading.Thread(target=worker) for _ in range(threads)]
    for t in pool:
        t.start()
    for t in pool:
        t.join()
    dt = time.perf_counter() - t0
    iters, steps = state["iters"], state["steps"]
    what = (f"{iters} single-iteration runs over tracks 0..{min(state['next'], pb.n_tracks) - 1}"
            if pb.n_tracks > 1 else f"{iters} iterations")
    return dict({"value": steps / dt, "unit": "steps/s", "cores": threads, "kind": "oracle",
                 "sample": f"{what}, {steps} steps{' (prefixes of T=' + str(cut) + ')' if cut < T0 else ''}, "
                           f"from the prior broadcast ({dt:.1f} s, {threads} thread{'s' if threads > 1 else ''}, "
                           f"gcc -O3 -march=native)"}, **host_cpu())


def binding_autotune(pb, stream, lin):
    from paper_2102_00514_amd import binding
    lanes, slots, _ = binding.smoother_autotune(pb, stream=stream, iters=5, lin=lin)
    return lanes, slots


def warm_start_section(weights: str, n_batch: int, n_single: int, lin: str = "taylor") -> dict:
    """Time to converge (trajectory change < 1e-6) from the prior broadcast vs
    from the learned initial trajectory, on held-out warm-start tracks
    (T = 4096): one batch of n_batch tracks in one handle, and n_single tracks
    one handle at a time (latency of a single track, best of 5 runs each)."""
    import numpy as np
    import torch
    from paper_2102_00514_amd import warmstart as W
    from paper_2102_00514_amd import workloads as wl
    stream = torch.cuda.current_stream().cuda_stream
    # inference in chunks of up to 16384 windows (about 1.7 GB of activations)
    net, cov, meta = W.load(weights, stream=stream, max_batch=16384)
    pb = wl.config_c4(0, n_batch, held_out=True)
    sched_batch = binding_autotune(pb, stream, lin)
    sched_single = binding_autotune(pb.track(0), stream, lin)
    W.time_to_converge(net, cov, pb.track(0), lin, schedule=sched_single)   # warm-up (kernels, allocator)
    batch = W._public(W.time_to_converge(net, cov, pb, lin, schedule=sched_batch, repeats=2, mfma=True))
    # the network's share of the learned start: inference and hand-over of the batch's trajectory
    d_y = torch.from_numpy(np.ascontiguousarray(pb.y)).cuda()
    net.set_tracks(pb.offsets)
    mean0 = torch.empty((pb.n_slots, pb.nx), dtype=torch.float64, device="cuda")
    net.trajectory(d_y.data_ptr(), mean0.data_ptr())
    torch.cuda.synchronize()
    for fast in (False, True):
        net.trajectory(d_y.data_ptr(), mean0.data_ptr(), mfma=fast)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            net.trajectory(d_y.data_ptr(), mean0.data_ptr(), mfma=fast)
        torch.cuda.synchronize()
        batch["inference_ms_" + ("bf16_mfma" if fast else "fp32")] = round((time.perf_counter() - t0) * 1e3 / 3, 3)
    batch["inference"] = "learned start inferred with BF16 products on the matrix cores (ws_trajectory_mfma)"
    batch["inference_chunk_windows"] = 16384
    del mean0, d_y
    rows = {"plain": [], "learned": []}
    for i in range(n_single):
        r = W.time_to_converge(net, cov, pb.track(i), lin, repeats=5, schedule=sched_single)
        for k in rows:
            rows[k].append((r[k]["ms_to_converge"], r[k]["iters_mean"]))
    single = {"tracks": n_single}
    for k, v in rows.items():
        ms = np.array([a if a is not None else np.nan for a, _ in v])
        single[k] = {"ms_median": float(np.nanmedian(ms)), "ms_mean": float(np.nanmean(ms)),
                     "iters_median": float(np.median([b for _, b in v])),
                     "converged": float(np.mean(np.isfinite(ms)))}
    single["speedup_median"] = single["plain"]["ms_median"] / single["learned"]["ms_median"]
    net.close()
    return {"weights": os.path.relpath(weights, ROOT), "lin": lin, "tol": 1e-6, "max_iter": 50, "T": wl.C4_T,
            "schedules": {"batch": list(sched_batch), "single_track": list(sched_single)},
            "trained_on": {k: meta.get(k) for k in ("tracks", "kept", "windows", "epochs", "train_s")},
            "batch": dict(batch, tracks=n_batch), "single_track": single}


def converge_section(pb, lin: str, schedule, tol: float = 1e-6, max_iter: int = 50, n_single: int = 64,
                     seed: int = 7) -> dict:
    """Converged-solution wall time of a batch: host wall time of
    smoother_iterate_until (tol on the largest change of each track, at most
    max_iter iterations) from the prior broadcast, for the whole batch in one
    handle (every track iterated until the last has converged), the same with
    converged tracks taken out of later iterations (freeze_converged), and a
    seeded sample of n_single tracks run one at a time on the same GPU, scaled
    to the batch by track count.  Each timed run starts from the prior
    broadcast after one untimed iteration (graph capture) has been undone."""
    import numpy as np
    import torch
    from paper_2102_00514_amd import binding
    stream = torch.cuda.current_stream().cuda_stream

    def timed_until(p, **kw):
        with binding.Smoother(p, stream=stream, n_iter=1, lin=lin, **kw) as sm:
            S, _, _ = sm.info()
            m0 = torch.empty((S, p.nx), dtype=torch.float64, device="cuda")
            sm.result_device(m0.data_ptr(), 0)
            sm.iterate(1, want_delta=False)                  # warm-up: graph capture
            sm.set_trajectory_device(m0.data_ptr(), 0)       # back to the prior broadcast (P0 per track)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run, first, _ = sm.iterate_until(tol, max_iter)
            wall = time.perf_counter() - t0
        return wall, run, first

    out = {"tol": tol, "max_iter": max_iter, "tracks": pb.n_tracks, "schedule": list(schedule), "lin": lin}
    for name, fz in (("batched", False), ("batched_freeze", True)):
        wall, run, first = timed_until(pb, tile_lanes=schedule[0], lane_slots=schedule[1], freeze_converged=fz)
        conv = first > 0
        it = np.where(conv, first, max_iter + 1)
        out[name] = {"ms": round(wall * 1e3, 3), "iterations_run": int(run), "converged": float(conv.mean()),
                     "iters_mean": float(it.mean()), "iters_median": float(np.median(it)),
                     "iters_p90": float(np.percentile(it, 90)), "iters_max_converged": int(first.max())}
        log(f"time to converge ({name}): {wall * 1e3:.1f} ms, {run} iterations, "
            f"{conv.mean() * 100:.1f}% converged, mean {it.mean():.1f} iterations")
    idx = np.sort(np.random.default_rng(seed).choice(pb.n_tracks, min(n_single, pb.n_tracks), replace=False))
    total = 0.0
    conv_single = 0
    for i in idx:
        wall, run, first = timed_until(pb.track(int(i)))
        total += wall
        conv_single += int(first[0] > 0)
    out["per_track"] = {"tracks_sampled": int(len(idx)), "ms_sample": round(total * 1e3, 3),
                        "ms_scaled_to_batch": round(total * 1e3 * pb.n_tracks / len(idx), 1),
                        "converged": conv_single / len(idx), "schedule": "default per track"}
    log(f"time to converge (one track at a time): {total * 1e3:.1f} ms for {len(idx)} tracks, "
        f"{total * 1e3 * pb.n_tracks / len(idx):.0f} ms scaled to {pb.n_tracks}")
    return out


def damping_section(n_batch: int, tol: float = 1e-6, max_iter: int = 50) -> dict:
    """Undamped iterations vs Levenberg-Marquardt passes with Marquardt's
    damping schedule (lambda0 = 1e-2, nu = 10), both from the prior broadcast,
    on the same held-out batch of warm-start tracks (T = 4096) in one handle:
    tracks converged within max_iter passes, mean passes of the converged
    tracks, wall time of the whole call, and how the final MAP objectives
    compare per track."""
    import time

    import numpy as np
    import torch
    from paper_2102_00514_amd import binding as Bn
    from paper_2102_00514_amd import workloads as wl
    stream = torch.cuda.current_stream().cuda_stream
    pb = wl.config_c4(0, n_batch, held_out=True)
    lanes, slots = binding_autotune(pb, stream, "taylor")
    with Bn.Smoother(pb, n_iter=1, lin="taylor", stream=stream, tile_lanes=lanes, lane_slots=slots) as sm:
        sm.iterate_lm(1e-2, 10.0, tol, 2)       # warm-up: kernels, graph capture
    res = {}
    for name in ("plain", "lm"):
        with Bn.Smoother(pb, n_iter=1, lin="taylor", stream=stream, tile_lanes=lanes, lane_slots=slots) as sm:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "plain":
                run, first, _ = sm.iterate_until(tol, max_iter)
            else:
                run, first, cost = sm.iterate_lm(1e-2, 10.0, tol, max_iter)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if name == "plain":
                cost = sm.objective()
        conv = first > 0
        res[name] = {"converged": float(conv.mean()), "passes_mean_converged": float(first[conv].mean()),
                     "passes_run": int(run), "ms": round(1e3 * wall, 3), "_cost": cost}
    lower = res["lm"]["_cost"] <= res["plain"]["_cost"] * (1 + 1e-9)
    out = {"tracks": n_batch, "T": wl.C4_T, "tol": tol, "max_iter": max_iter, "lambda0": 1e-2, "nu": 10.0,
           "schedule": [lanes, slots]}
    for k in ("plain", "lm"):
        out[k] = {a: b for a, b in res[k].items() if not a.startswith("_")}
    out["lm_objective_not_above_plain"] = float(lower.mean())
    return out


def c2_sweep(args) -> None:
    """T = 2^10..2^15 (prefixes of the seed-0 track): ms per iteration of the
    GPU parallel path (Taylor and cubature, FP64 and FP32), of the GPU
    sequential path (one lane runs the Kalman filter and RTS smoother), and
    of the CPU oracle (one thread, Taylor), each at its autotuned schedule.
    Prints one JSON line whose value is the parallel FP64 Taylor rate at the
    longest T."""
    import torch
    from paper_2102_00514_amd import binding
    from paper_2102_00514_amd import workloads as wl
    oracle = native_oracle()
    stream = torch.cuda.current_stream()
    rows = []
    cases = [("taylor", "f64", "parallel"), ("cubature", "f64", "parallel"), ("taylor", "f32", "parallel"),
             ("cubature", "f32", "parallel"), ("taylor", "f64", "sequential"), ("cubature", "f64", "sequential")]
    for e in range(10, 16):
        T = 2 ** e
        pb = wl.config_c2(T)
        row = {"T": T}
        for lin, prec, scan in cases:
            kw = dict(lin=lin, precision=prec, scan=scan)
            if scan == "parallel":
                lanes, slots, _ = binding.smoother_autotune(pb, stream=stream.cuda_stream, iters=5, **kw)
                kw.update(tile_lanes=lanes, lane_slots=slots)
            with binding.Smoother(pb, stream=stream.cuda_stream, n_iter=1000, **kw) as sm:
                sm.iterate(3, want_delta=False)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                k = 20 if scan == "parallel" else 3
                torch.cuda.synchronize()
                a.record(stream)
                sm.iterate(k, want_delta=False)
                b.record(stream)
                torch.cuda.synchronize()
                row[f"{scan}_{lin}_{prec}_ms"] = round(a.elapsed_time(b) / k, 4)
        t0 = time.perf_counter()
        reps = 0
        while True:
            oracle.smoother(pb, 1, "taylor", filtered=False)
            reps += 1
            if time.perf_counter() - t0 > 0.5:
                break
        row["cpu_oracle_taylor_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
        log(json.dumps(row))
        rows.append(row)
    top = rows[-1]
    ms = top["parallel_taylor_f64_ms"]
    print(json.dumps({
        "metric": METRIC, "value": round(top["T"] / (ms * 1e-3), 1), "unit": "steps/s", "n_gpus": 1,
        "steps": 20, "warmup": 3, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "coordinated-turn + 2 bearings, T = 2^10..2^15 prefixes of one track; "
                               "GPU parallel / GPU sequential / CPU oracle (1 thread)", "parallelism": "1 GPU"},
        "sweep": rows}), flush=True)


WORKLOADS = {
    "c2": "coordinated-turn + 2 bearings, T={T}, single track",
    "c3": "4096 coordinated-turn tracks, T_i ~ U{{100..8192}}, 2 bearings, one ragged batch",
    "c5": "4 stacked coordinated-turn targets (nx=20), 8 bearings, T={T}, single track",
    "c5batch": "256 tracks of 4 stacked coordinated-turn targets (nx=20), 8 bearings, T_i ~ U{{1024..65536}}, "
               "one ragged batch",
}
DEFAULT_LIN = {"c2": "taylor", "c3": "cubature", "c5": "unscented", "c5batch": "unscented"}


def make_workload(name: str, T: int = 0):
    from paper_2102_00514_amd import workloads as wl
    if name == "c2":
        pb = wl.config_c2(T or 2 ** 15)
    elif name == "c3":
        pb = wl.config_c3()
    elif name == "c5":
        pb = wl.config_c5_single(T or 2 ** 16)
    else:
        pb = wl.config_c5_batch()
    return pb, WORKLOADS[name].format(T=int(pb.offsets[1]))


def measure(name: str, pb, desc: str, lin: str, precision: str, steps: int, warmup: int, profile_iters: int,
            tile_lanes: int = 0, lane_slots: int = 0, autotune: bool = True, check: bool = True,
            form: str = "covariance") -> dict:
    """Times `steps` iterations of the captured iteration graph on resident
    inputs (HIP events on the handle's stream), then a separate pass of
    `profile_iters` iterations with HIP events around every kernel launch for
    the roofline of the dominant kernel.  With check, the trajectory after the
    timed iterations is checked to be finite with symmetric covariances."""
    import numpy as np
    import torch
    from paper_2102_00514_amd import binding
    T = int(pb.offsets[-1])            # smoothed steps per iteration (all tracks)
    dense = pb.nx == 20 and lin != "taylor"
    stream = torch.cuda.current_stream()
    tuned = None
    if autotune and not tile_lanes and not lane_slots:
        lanes_t, slots_t, ms_t = binding.smoother_autotune(pb, stream=stream.cuda_stream,
                                                           iters=10 if pb.n_slots < 2 ** 20 else 2, lin=lin,
                                                           precision=precision, form=form)
        tuned = {"tile_lanes": lanes_t, "lane_slots": slots_t, "ms_per_iter": round(ms_t, 6)}
        log(f"{name}: autotuned schedule: {lanes_t} lanes x {slots_t} slots ({ms_t * 1e3:.1f} us/iteration)")
        tile_lanes, lane_slots = lanes_t, slots_t
    sm = binding.Smoother(pb, stream=stream.cuda_stream, n_iter=warmup + steps + profile_iters, lin=lin,
                          precision=precision, tile_lanes=tile_lanes, lane_slots=lane_slots, form=form)
    S, _, dev_bytes = sm.info()
    lanes, slots, tiles = sm.schedule()
    log(f"workload {name}: steps={T} slots={S} lin={lin} precision={precision} device_bytes={dev_bytes} "
        f"schedule: {tiles} tiles x {lanes} lanes x {slots} slots")

    sm.iterate(warmup, want_delta=False)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t_start.record(stream)
    sm.iterate(steps, want_delta=False)
    t_stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_stop)
    ms_per_step = ms_total / steps
    value = T / (ms_per_step * 1e-3)
    log(f"{name}: timed {steps} iterations: {ms_total:.3f} ms (events), {wall * 1e3:.3f} ms (host wall); "
        f"{ms_per_step * 1e3:.1f} us/iteration")

    checked = None
    if check:
        # the iterate after the timed iterations: finite, symmetric covariances.
        # A track whose iterate stops being finite is reported failed by the
        # library (its change statistic is NaN); every other track must hold a
        # finite, symmetric trajectory, and no failure may go unreported.
        dt = torch.float64 if precision == "f64" else torch.float32
        mean = torch.empty((S, pb.nx), dtype=dt, device="cuda")
        cov = torch.empty((S, pb.nx, pb.nx), dtype=dt, device="cuda")
        sm.result_device(mean.data_ptr(), cov.data_ptr())
        torch.cuda.synchronize()
        not_finite = np.zeros(S, dtype=bool)
        not_symmetric = np.zeros(S, dtype=bool)
        for a in range(0, S, 1 << 20):          # bounded temporaries next to a large plan
            c = cov[a:a + (1 << 20)]
            m = mean[a:a + (1 << 20)]
            nf = ~torch.isfinite(m).all(dim=1) | ~torch.isfinite(c).all(dim=2).all(dim=1)
            ns = (c != c.transpose(1, 2)).any(dim=2).any(dim=1) & ~nf
            not_finite[a:a + len(c)] = nf.cpu().numpy()
            not_symmetric[a:a + len(c)] = ns.cpu().numpy()
        del cov
        del mean
        deltas = sm.track_deltas()
        failed = ~np.isfinite(deltas)
        slot_failed = np.repeat(failed, np.diff(pb.slot_offsets()))
        ok_f = not bool((not_finite & ~slot_failed).any())
        ok_s = not bool(not_symmetric.any())
        checked = {"finite": ok_f, "symmetric": ok_s, "failed_tracks": int(failed.sum()),
                   "deltas_finite": not bool(failed.any()), "iterations_done": warmup + steps}
        if failed.any():
            checked["failed_track_ids"] = [int(i) for i in np.nonzero(failed)[0][:16]]
        log(f"{name}: trajectory after the timed iterations: {checked}")
        assert ok_f and ok_s, f"{name}: non-finite or asymmetric trajectory outside the tracks reported failed"

    # per-kernel durations from HIP events around each launch (separate pass;
    # each launch repeated 8 times between its events, the mean taken)
    prof = sm.profile(profile_iters, repeat=PROFILE_REPEAT)
    torch.cuda.synchronize()
    word = 8 if precision == "f64" else 4
    scan_b = scan_bytes_per_slot(pb.nx, word)
    rows = []
    for kname, (launches, tot_ms, positions) in prof.items():
        per_iter_us = tot_ms * 1e3 / profile_iters
        if dense:      # per position: floating-point operations
            upp = dense_flops_per_position(kname, pb.nx, pb.ny)
            rate = upp * positions / (tot_ms * 1e-3) / 1e12 if tot_ms > 0 else 0.0
            dpp = upp
        else:          # per position: the method's bytes; the design's beside them
            upp = scan_b[KERNEL_SCAN[kname]] if kname in KERNEL_SCAN else 0.0
            dpp = design_bytes_per_position(kname, pb.nx, pb.ny, lin, word, slots)
            rate = upp * positions / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
        rows.append((per_iter_us, kname, launches, tot_ms, positions, upp, rate, dpp))
    rows.sort(reverse=True)
    unit_pp, unit_rate = ("flop/pos", "TFLOP/s") if dense else ("B/pos", "GB/s")
    log(f"{'kernel':28s} {'us/iter':>9s} {'launches':>8s} {'avg us':>9s} {unit_pp:>9s} {unit_rate:>8s} "
        f"{'design B/pos' if not dense else '':>12s}")
    for per_iter_us, kname, launches, tot_ms, positions, upp, rate, dpp in rows:
        log(f"{kname:28s} {per_iter_us:9.2f} {launches:8d} {tot_ms * 1e3 / launches:9.2f} {upp:9.0f} {rate:8.2f} "
            f"{'' if dense else f'{dpp:12.0f}'}")
    sum_us = sum(r[0] for r in rows)
    log(f"{name}: sum of kernel time per iteration: {sum_us:.1f} us (vs {ms_per_step * 1e3:.1f} us end to end)")
    dom = rows[0]
    avg_launch_s = dom[3] * 1e-3 / dom[2]
    units_per_launch = dom[5] * dom[4] / dom[2]
    iteration = None
    if dense:
        achieved = units_per_launch / avg_launch_s / 1e12
        # the full-state engine's linearisation computes in FP64 at either precision
        peak = FP32_VECTOR_PEAK_TFLOPS if precision == "f32" and dom[1] != "dn_linearize" else FP64_VECTOR_PEAK_TFLOPS
        roofline = {"bound": "alu", "kernel": dom[1], "achieved": round(achieved, 4),
                    "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 6), "traffic": None,
                    "avg_launch_us": round(avg_launch_s * 1e6, 3), "flops_per_launch": int(units_per_launch)}
    else:
        achieved = units_per_launch / avg_launch_s / 1e9
        traffic = measured_traffic(f"{dom[1]}|T={T}|{lin}|{precision}" + ("|sqrt" if form == "sqrt" else ""))
        design = dom[7] * dom[4] / dom[2]
        roofline = {"bound": "hbm", "kernel": dom[1], "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                    "traffic": None if traffic is None else int(traffic),
                    "avg_launch_us": round(avg_launch_s * 1e6, 3), "bytes_per_launch": int(units_per_launch),
                    "bytes_per_slot": dom[5], "slots_per_launch": int(dom[4] / dom[2]),
                    "design_bytes_per_launch": int(design),
                    "traffic_over_algorithmic": None if traffic is None else round(traffic / units_per_launch, 4)}
        it_bytes = scan_b["iteration"] * S
        iteration = {"bytes_per_slot": scan_b["iteration"], "bytes": int(it_bytes),
                     "achieved_GBs": round(it_bytes / (ms_per_step * 1e-3) / 1e9, 3),
                     "frac": round(it_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 6)}
    res = {"value": round(value, 1), "ms_per_step": round(ms_per_step, 6), "steps": steps, "warmup": warmup,
           "dtype": precision, "S": S, "T": T, "tracks": pb.n_tracks, "nx": pb.nx, "ny": pb.ny, "lin": lin,
           "desc": desc, "schedule": {"tiles": tiles, "lanes_per_tile": lanes, "slots_per_lane": slots,
                                      "autotuned": tuned},
           "roofline": roofline, "iteration_roofline": iteration, "checked": checked,
           "kernels_us_per_iter": {r[1]: round(r[0], 3) for r in rows}, "_sm": sm}
    return res


def binding_handle_for_filter(pb, args):
    import torch
    from paper_2102_00514_amd import binding
    return binding.Smoother(pb, stream=torch.cuda.current_stream().cuda_stream, n_iter=1, lin=args.lin,
                            precision=args.precision, tile_lanes=args.tile_lanes, lane_slots=args.lane_slots)


def extra_line(name: str, r: dict, cpu) -> dict:
    return {"workload": r["desc"], "lin": r["lin"], "dtype": r["dtype"], "value": r["value"], "unit": "steps/s",
            "ms_per_step": r["ms_per_step"], "steps": r["steps"], "warmup": r["warmup"], "slots": r["S"],
            "schedule": r["schedule"], "roofline": r["roofline"], "iteration_roofline": r["iteration_roofline"],
            "checked": r["checked"], "kernels_us_per_iter": r["kernels_us_per_iter"], "cpu_baseline": cpu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c5", "c5batch", "c2sweep"],
                    help="c2: one track, T=2^15 (default); c3: 4096 ragged tracks; c5: four stacked targets, "
                         "T=2^16; c5batch: 256 ragged stacked tracks, T_i in [1024, 2^16]")
    ap.add_argument("--T", type=int, default=0, help="track length (c2: 2^15, c5: 2^16)")
    ap.add_argument("--lin", default=None, choices=["taylor", "cubature", "unscented"],
                    help="default: taylor (c2), cubature (c3), unscented (c5)")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--form", default="covariance", choices=["covariance", "sqrt"],
                    help="element form: the paper's covariance form or lower-triangular factors")
    ap.add_argument("--profile-iters", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain copy kernel of 256 MiB in, 256 MiB out (counter calibration)")
    ap.add_argument("--tile-lanes", type=int, default=0, help="scan schedule override (64 or 256)")
    ap.add_argument("--lane-slots", type=int, default=0, help="scan schedule override (1..32)")
    ap.add_argument("--no-autotune", action="store_true", help="use the default schedule instead of the autotuner's")
    ap.add_argument("--warm-start-weights", default=os.path.join(ROOT, "paper_2102_00514_amd", "weights",
                                                                 "warmstart_ieks.npz"))
    ap.add_argument("--warm-start-tracks", type=int, default=512, help="held-out tracks in the batch comparison")
    ap.add_argument("--warm-start-single", type=int, default=32, help="held-out tracks timed one at a time")
    ap.add_argument("--no-warm-start", action="store_true")
    ap.add_argument("--no-damping", action="store_true", help="skip the Levenberg-Marquardt comparison")
    ap.add_argument("--damping-tracks", type=int, default=512, help="held-out tracks in the damping comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="c2 only: skip the 4096-track batch and the nx=20 track timed beside the headline")
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the converged-solution wall times of the batch (c3, and the extra c3 line)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the smoother's single-track "
                          "workload is not sharded across GPUs", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # a plain elementwise copy with known traffic, for scaling hardware byte counters
        src = torch.full((32 * 2 ** 20,), 1.0, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 B read, 268435456 B written by one elementwise kernel")
        del src, dst
    if args.workload == "c2sweep":
        c2_sweep(args)
        return
    if args.lin is None:
        args.lin = DEFAULT_LIN[args.workload]
    pb, desc = make_workload(args.workload, args.T)
    if args.workload != "c2":
        args.no_warm_start = True
        args.no_damping = True
        args.no_extra = True
    r = measure(args.workload, pb, desc, args.lin, args.precision, args.steps, args.warmup, args.profile_iters,
                args.tile_lanes, args.lane_slots, autotune=not args.no_autotune, form=args.form)
    sm = r.pop("_sm")
    converge = None
    if args.workload == "c3" and not args.no_converge:
        sch = r["schedule"]
        sm.close()
        converge = converge_section(pb, args.lin, (sch["lanes_per_tile"], sch["slots_per_lane"]))
        sm = binding_handle_for_filter(pb, args)
    dense = pb.nx == 20 and args.lin != "taylor"
    filter_pass = None
    if not dense:
        # filtering pass with the log marginal likelihood at the current
        # trajectory (host wall per call, including the per-track copy back)
        for _ in range(3):
            sm.filter(moments=False)
        n_f = 20
        w0 = time.perf_counter()
        for _ in range(n_f):
            _, _, ll = sm.filter(moments=False)
        ms_f = (time.perf_counter() - w0) * 1e3 / n_f
        filter_pass = {"ms_per_pass": round(ms_f, 4), "loglik_track0": float(ll[0]),
                       "timing": "host wall per call, log-likelihood copied to the host"}
        log(f"filtering pass with log-likelihood: {ms_f * 1e3:.1f} us per call")
    sm.close()
    del pb

    cpu = None
    if not args.no_cpu:
        pb, _ = make_workload(args.workload, args.T)
        threads = 1 if pb.n_tracks == 1 else (os.cpu_count() or 1)
        cpu = cpu_baseline(pb, args.lin, args.cpu_seconds, threads=threads)
        log(f"cpu oracle: {cpu['value']:.4g} steps/s ({cpu['sample']})")
        del pb

    extra = {}
    if not args.no_extra:
        # the other two headline shapes, timed in the same run (fewer iterations),
        # the full-state shape's FP32 variant, and the full-state batch (256
        # tracks, 161 GB of device memory; its fixed default schedule, since
        # trying five would build five such plans)
        for key, name, prec, steps, warmup in (("c3", "c3", "f64", 5, 2), ("c5", "c5", "f64", 5, 2),
                                               ("c5_f32", "c5", "f32", 5, 2), ("c5batch", "c5batch", "f64", 3, 1)):
            pbx, descx = make_workload(name)
            rx = measure(name, pbx, descx, DEFAULT_LIN[name], prec, steps, warmup, 1 if key == "c5batch" else 2,
                         autotune=key != "c5batch")
            rx.pop("_sm").close()
            conv = None
            if key == "c3" and not args.no_converge:     # the batch the time-to-converge comparison is on
                sch = rx["schedule"]
                conv = converge_section(pbx, DEFAULT_LIN[name], (sch["lanes_per_tile"], sch["slots_per_lane"]))
            cpux = None
            if not args.no_cpu and prec == "f64":
                threads = 1 if pbx.n_tracks == 1 else (os.cpu_count() or 1)
                cpux = cpu_baseline(pbx, DEFAULT_LIN[name], min(args.cpu_seconds, 8.0), threads=threads)
                log(f"{name} cpu oracle: {cpux['value']:.4g} steps/s ({cpux['sample']})")
            extra[key] = extra_line(name, rx, cpux)
            if conv is not None:
                extra[key]["time_to_converge"] = conv
            del pbx
            torch.cuda.empty_cache()

    warm = None
    if not args.no_warm_start and os.path.exists(args.warm_start_weights):
        warm = warm_start_section(args.warm_start_weights, args.warm_start_tracks, args.warm_start_single)
        log(f"time to converge (1e-6), held-out batch of {args.warm_start_tracks}: "
            f"plain {warm['batch']['plain']['iters_mean']:.2f} iterations (mean), "
            f"learned {warm['batch']['learned']['iters_mean']:.2f}; single track median "
            f"{warm['single_track']['plain']['ms_median']:.3f} ms plain vs "
            f"{warm['single_track']['learned']['ms_median']:.3f} ms learned")

    damping = None
    if not args.no_damping:
        damping = damping_section(args.damping_tracks)
        log(f"held-out batch of {args.damping_tracks}, prior start: undamped converged "
            f"{damping['plain']['converged']:.3f} ({damping['plain']['passes_mean_converged']:.2f} passes, "
            f"{damping['plain']['ms']:.1f} ms), Levenberg-Marquardt {damping['lm']['converged']:.3f} "
            f"({damping['lm']['passes_mean_converged']:.2f} passes, {damping['lm']['ms']:.1f} ms)")

    out = {
        "metric": METRIC, "value": r["value"], "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"{desc} ({r['S']} slots), "
                               f"{'IEKS (Taylor)' if args.lin == 'taylor' else args.lin + ' SLR'}, "
                               f"one iteration per step",
                   "T": r["T"], "tracks": r["tracks"], "nx": r["nx"], "ny": r["ny"], "lin": args.lin,
                   "form": args.form, "parallelism": "time-axis scan, 1 GPU", "schedule": r["schedule"]},
        "roofline": r["roofline"],
        "iteration_roofline": r["iteration_roofline"],
        "cpu_baseline": cpu,
        "checked": r["checked"],
        "kernels_us_per_iter": r["kernels_us_per_iter"],
        "time_to_converge": converge,
        "extra": extra or None,
        "warm_start": warm,
        "damping": damping,
        "filter_pass": filter_pass,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
