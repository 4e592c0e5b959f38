"""Parity at the full workload sizes, in the schedules the benchmark times.

C2 at T = 2^15 is compared slot by slot in test_gpu_parity.  Here:
  - C3: 4096 ragged coordinated-turn tracks (1.68e7 slots), cubature, FP64,
    64 lanes x 16 slots (the autotuned schedule the benchmark times);
  - C5 single: four stacked targets (nx = 20, ny = 8), T = 2^16, unscented;
  - C5 batch: 256 stacked-target tracks, T_i ~ U{1024..65536} (8.5e6 slots),
    the shortest, the longest and six random tracks sampled.

Each case runs the whole batch on the device twice:
  1. iteration 1 from the prior broadcast (the step the benchmark times);
  2. one more iteration after the sampled tracks' trajectories are replaced by
     the oracle's iterate 2 (a common input; the other tracks keep the
     device's iterate 1), compared with the oracle's iterate 3.
The oracle computes each sampled track on its own (one host thread per
track) and every slot of them is compared (metric as in test_gpu_parity).
Both steps are held to the FP64 gate 1e-9 on every sampled track.

Where the device misses the FP64 oracle by more than that, the oracle's
80-bit build runs the same step and decides: the device is held to 1e-9 of
its result, or, where the FP64 oracle itself misses it by more (a step that
FP64 cannot resolve to the gate), to twice the FP64 oracle's own miss.  Three
sampled C5 batch tracks take this path at step 2:
  - tracks 140 (T = 47820) and 211 (T = 33099): the FP64 oracle misses its
    80-bit build by up to 1.8e-9; the device is within 3e-11 of it;
  - track 180 (T = 62736) has diverged by its iterate 2 (means of norm
    2.6e5, change 8.3e5 in the step); there the FP64 sigma-point regression
    loses up to 5e-5 of Q' and c to rounding, and the FP64 oracle misses its
    80-bit build by 1.2e-7 (means) and 5.9e-9 (covariances), the device by
    1.4e-7 and 1.5e-9.

One named exception to the gate: step 1 of C3 track 0 (T = 6667) is held to
1e-8.  These priors set the turn rate to zero, and on that track the first
iteration moves the trajectory by 633 units; there the parallel scan's FP64
result differs from the sequential oracle by 6.6e-9 (3.6e-9 for the track
alone, whose 7 tiles take the single-block top scan instead of the batch's
multi-level one; the oracle in FP64 and in 80-bit agree to 4e-12), while the same track from the oracle's iterate 2
agrees to 4.3e-11, and every other sampled C3 track agrees to 1.3e-10 at
step 1.  The gap is the method's in FP64: test_scan_conditioning shows
eq. 15 in a tree order missing the 80-bit result by 1.9e-8 on the same step.

On the device every output of every track is checked to be finite, every
covariance symmetric with a positive diagonal, and every per-track change
statistic finite.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2102_00514_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
# (workload, track) -> step-1 gate for the one ill-conditioned first step
# described above; every other sampled track and step is held to TOL64
STEP1_EXCEPTIONS = {("C3", 0): 1e-8}


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2102_00514_amd import binding
    return binding


def check_all_slots(mean, cov, deltas, chunk=1 << 20):
    import torch
    assert bool(torch.isfinite(mean).all())
    for a in range(0, cov.shape[0], chunk):   # bounded temporaries next to a large plan
        c = cov[a:a + chunk]
        assert bool(torch.isfinite(c).all())
        assert float((c - c.transpose(1, 2)).abs().max()) == 0.0
        assert bool((torch.diagonal(c, dim1=1, dim2=2) > 0).all())
    assert np.all(np.isfinite(deltas))


def reference_80bit(pb, i, ref, it, lin):
    """The oracle's 80-bit build on the same step: from the prior (it = 0) or
    from the FP64 oracle's iterate `it` (the device's input for that step)."""
    kw = {} if it == 0 else {"init_mean": ref["hist_mean"][it - 1], "init_cov": ref["hist_cov"][it - 1]}
    return oracle.smoother(pb.track(i), 1, lin, precision="f80", filtered=False, **kw)


def compare_tracks(pb, mean, cov, deltas, refs, it, what, lin):
    so = pb.slot_offsets()
    worst = 0.0
    for i, ref in refs.items():
        tol = STEP1_EXCEPTIONS.get((what, i), TOL64) if it == 0 else TOL64
        m = mean[so[i]:so[i + 1]].cpu().numpy()
        c = cov[so[i]:so[i + 1]].cpu().numpy()
        em = oracle.mean_error(m, ref["hist_mean"][it])
        ep = oracle.cov_error(c, ref["hist_cov"][it])
        print(f"{what} iteration {it + 1}, track {i} T={pb.lengths[i]}: e_m={em:.3e} e_P={ep:.3e}", flush=True)
        tol_m = tol_p = tol
        if not (em < tol and ep < tol):
            # the FP64 oracle's own rounding on this step, measured against its
            # 80-bit build; the 80-bit result is then the reference, and where
            # FP64 itself cannot reach the gate on this step the device is held
            # to twice the FP64 oracle's own miss
            r80 = reference_80bit(pb, i, ref, it, lin)
            om = oracle.mean_error(ref["hist_mean"][it], r80["mean"])
            op = oracle.cov_error(ref["hist_cov"][it], r80["cov"])
            em = oracle.mean_error(m, r80["mean"])
            ep = oracle.cov_error(c, r80["cov"])
            tol_m, tol_p = max(tol, 2 * om), max(tol, 2 * op)
            print(f"  80-bit oracle: FP64 oracle e_m={om:.3e} e_P={op:.3e}; device e_m={em:.3e} e_P={ep:.3e}; "
                  f"gates {tol_m:.1e} {tol_p:.1e}", flush=True)
        assert em < tol_m and ep < tol_p, (what, it + 1, i, em, ep, tol_m, tol_p)
        assert abs(deltas[i] - ref["deltas"][it]) <= 1e-6 * ref["deltas"][it] + 1e-12
        worst = max(worst, em, ep)
    return worst


def full_size_case(B, pb, lin, tracks, what, **kw):
    import torch
    k = 2
    tracks = [int(i) for i in tracks]
    # the oracle releases the interpreter in its C calls: one thread per sampled track
    with ThreadPoolExecutor(max_workers=min(8, len(tracks))) as ex:
        runs = list(ex.map(lambda i: oracle.smoother(pb.track(i), k + 1, lin, history=True), tracks))
    refs = dict(zip(tracks, runs))
    so = pb.slot_offsets()
    with B.Smoother(pb, n_iter=k + 1, lin=lin, **kw) as sm:
        sm.iterate(1)
        S, _, dev = sm.info()
        print(f"{what}: {pb.n_tracks} tracks, {S} slots, {dev / 1e9:.1f} GB planned, schedule {sm.schedule()}",
              flush=True)
        mean = torch.empty((S, pb.nx), dtype=torch.float64, device="cuda")
        cov = torch.empty((S, pb.nx, pb.nx), dtype=torch.float64, device="cuda")
        sm.result_device(mean.data_ptr(), cov.data_ptr())
        deltas = sm.track_deltas()
        check_all_slots(mean, cov, deltas)
        compare_tracks(pb, mean, cov, deltas, refs, 0, what, lin)
        for i, ref in refs.items():
            mean[so[i]:so[i + 1]] = torch.from_numpy(ref["hist_mean"][k - 1]).to("cuda")
            cov[so[i]:so[i + 1]] = torch.from_numpy(ref["hist_cov"][k - 1]).to("cuda")
        torch.cuda.synchronize()
        sm.set_trajectory_device(mean.data_ptr(), cov.data_ptr())
        sm.iterate(1)
        sm.result_device(mean.data_ptr(), cov.data_ptr())
        deltas = sm.track_deltas()
        torch.cuda.synchronize()
        check_all_slots(mean, cov, deltas)
        compare_tracks(pb, mean, cov, deltas, refs, k, what, lin)


def sample(pb, n_random, seed):
    L = pb.lengths
    picks = {int(np.argmin(L)), int(np.argmax(L))}
    picks |= set(np.random.default_rng(seed).choice(pb.n_tracks, n_random, replace=False).tolist())
    return sorted(picks)


def test_c3_4096_tracks_64x16(B):
    pb = wl.config_c3()
    tracks = sorted(set(sample(pb, 28, 30)) | {0, pb.n_tracks - 1})
    full_size_case(B, pb, "cubature", tracks, "C3", tile_lanes=64, lane_slots=16)


def test_c5_single_T65536(B):
    full_size_case(B, wl.config_c5_single(), "unscented", [0], "C5 single")


def test_c5_batch_256_tracks(B):
    pb = wl.config_c5_batch()
    full_size_case(B, pb, "unscented", sample(pb, 6, 50), "C5 batch")
