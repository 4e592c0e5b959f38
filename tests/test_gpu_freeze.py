"""Converged tracks taken out of later iterations (sm_problem.freeze_converged).

smoother_iterate_until with freeze_converged stops iterating a track once its
change statistic is below tol: its slots then hold padding elements, which
restart both scans, and tiles whose tracks have all converged are skipped.
Every other track must come out exactly as without freezing, and each
frozen track must hold the oracle's iterate of the iteration at which it
converged.  Gates as in test_gpu_parity (FP64 1e-9).
"""
import numpy as np
import pytest

import oracle
from paper_2102_00514_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2102_00514_amd import binding
    return binding


def batch():
    # lengths chosen so that some tracks span many 64-slot tiles; the seeds
    # give different numbers of iterations to converge
    return wl.concat_tracks([wl.ct_bearings(T, seed=80 + T) for T in (900, 7, 1, 300, 2000, 40, 130)], "ragged")


def run_until(B, pb, lin, tol, max_iter, freeze, **kw):
    with B.Smoother(pb, n_iter=1, lin=lin, freeze_converged=freeze, **kw) as sm:
        run, first, ok = sm.iterate_until(tol, max_iter)
        mean, cov = sm.result()
    return run, first, mean, cov


@pytest.mark.parametrize("lin,lanes,slots,form", [("taylor", 64, 1, "covariance"), ("taylor", 64, 8, "covariance"),
                                                  ("cubature", 256, 2, "covariance"), ("taylor", 64, 4, "sqrt")])
def test_frozen_tracks_hold_their_converged_iterate(B, lin, lanes, slots, form):
    pb = batch()
    tol = 1e-8
    run_f, first_f, mean, cov = run_until(B, pb, lin, tol, 60, True, tile_lanes=lanes, lane_slots=slots, form=form)
    run_p, first_p, _, _ = run_until(B, pb, lin, tol, 60, False, tile_lanes=lanes, lane_slots=slots, form=form)
    print(f"{lin} {lanes}x{slots} {form}: runs {run_f}/{run_p}, first {list(first_f)}", flush=True)
    # the same iterations to converge with and without freezing
    assert run_f == run_p and np.array_equal(first_f, first_p)
    # tracks converged at different iterations, and a frozen track held a
    # whole tile while others still ran (so that tile was skipped)
    conv = first_f > 0
    assert conv.sum() >= pb.n_tracks - 1 and len(set(first_f[conv].tolist())) > 1
    so = pb.slot_offsets()
    per_tile = lanes * slots
    whole = [i for i in range(pb.n_tracks)
             if conv[i] and first_f[i] < run_f and (so[i + 1] // per_tile) > -(-so[i] // per_tile)]
    assert whole, "no frozen track held a whole tile"
    for i in range(pb.n_tracks):
        sl = slice(so[i], so[i + 1])
        assert np.all(np.isfinite(mean[sl])) and np.all(np.isfinite(cov[sl]))
        if not conv[i]:
            continue        # iterated to the cap without converging: not a parity point
        ref = oracle.smoother(pb.track(i), int(first_f[i]), lin)
        sl = slice(so[i], so[i + 1])
        em = oracle.mean_error(mean[sl], ref["mean"])
        ep = oracle.cov_error(cov[sl], ref["cov"])
        assert em < TOL64 and ep < TOL64, (i, int(first_f[i]), em, ep)


def test_iterations_after_the_call_run_every_track(B):
    pb = batch()
    with B.Smoother(pb, n_iter=1, freeze_converged=True, tile_lanes=64, lane_slots=1) as sm:
        run, first, _ = sm.iterate_until(1e-8, 60)
        sm.iterate(1, want_delta=False)
        mean, cov = sm.result()
        deltas = sm.track_deltas()
    assert np.all(np.isfinite(deltas))
    so = pb.slot_offsets()
    for i in range(pb.n_tracks):
        ref = oracle.smoother(pb.track(i), int(first[i]) + 1, "taylor")
        sl = slice(so[i], so[i + 1])
        em = oracle.mean_error(mean[sl], ref["mean"])
        ep = oracle.cov_error(cov[sl], ref["cov"])
        assert em < TOL64 and ep < TOL64, (i, em, ep)
        assert abs(deltas[i] - ref["deltas"][-1]) <= 1e-6 * ref["deltas"][-1] + 1e-12


def test_failed_track_is_taken_out(B):
    import torch
    pb = batch()
    L = pb.lengths
    so = pb.slot_offsets()
    mean = torch.from_numpy(np.repeat(pb.m0, L + 1, axis=0)).to("cuda")
    cov = torch.from_numpy(np.repeat(pb.P0, L + 1, axis=0)).to("cuda")
    bad = 4
    mean[so[bad] + L[bad] // 2, 0] = float("nan")
    torch.cuda.synchronize()
    with B.Smoother(pb, n_iter=1, freeze_converged=True, tile_lanes=64, lane_slots=2) as sm:
        sm.set_trajectory_device(mean.data_ptr(), cov.data_ptr())
        run, first, ok = sm.iterate_until(1e-8, 60)
        m, c = sm.result()
    assert not ok and first[bad] == 0
    # every other track converges and holds the oracle's iterate of that iteration
    for i in range(pb.n_tracks):
        if i == bad:
            continue
        assert first[i] > 0
        sl = slice(so[i], so[i + 1])
        ref = oracle.smoother(pb.track(i), int(first[i]), "taylor")
        em = oracle.mean_error(m[sl], ref["mean"])
        ep = oracle.cov_error(c[sl], ref["cov"])
        assert em < TOL64 and ep < TOL64, (i, int(first[i]), em, ep)
