"""A failed track stays in its own slots.

One track of a ragged batch gets a non-finite linearisation point (written on
the device through smoother_set_trajectory_device, as a broken caller-supplied
start would).  Its change statistic comes back NaN and the call reports the
non-finite iterate, while every other track -- before it (the smoothing scan
runs backward) and after it (the filtering scan runs forward) -- still equals
the oracle's iteration from the same input: the prior and end elements that
open and close each track restart both scans (Section 4), also when the
operand on the other side of them is NaN.
"""
import numpy as np
import pytest

import oracle
from paper_2102_00514_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2102_00514_amd import binding
    return binding


def run_with_failed_track(B, pb, bad, lin, precision="f64", **kw):
    """One iteration from the prior broadcast, with a NaN in track `bad`."""
    import torch
    dt = torch.float64 if precision == "f64" else torch.float32
    L = pb.lengths
    mean = torch.from_numpy(np.repeat(pb.m0, L + 1, axis=0)).to("cuda", dt)
    cov = torch.from_numpy(np.repeat(pb.P0, L + 1, axis=0)).to("cuda", dt)
    so = pb.slot_offsets()
    mean[so[bad] + L[bad] // 2, 0] = float("nan")
    torch.cuda.synchronize()
    with B.Smoother(pb, n_iter=1, lin=lin, precision=precision, **kw) as sm:
        sm.set_trajectory_device(mean.data_ptr(), cov.data_ptr())
        delta, _ = sm.iterate(1)
        m, c = sm.result()
        deltas = sm.track_deltas()
    return delta, m, c, deltas


def check_others(pb, bad, lin, delta, m, c, deltas, tol):
    assert np.isnan(delta)
    assert np.isnan(deltas[bad])
    so = pb.slot_offsets()
    for i in range(pb.n_tracks):
        if i == bad:
            continue
        ref = oracle.smoother(pb.track(i), 1, lin)
        sl = slice(so[i], so[i + 1])
        em = oracle.mean_error(m[sl], ref["mean"])
        ep = oracle.cov_error(c[sl], ref["cov"])
        print(f"failed track {bad}: track {i} T={pb.lengths[i]} e_m={em:.2e} e_P={ep:.2e}", flush=True)
        assert em < tol and ep < tol, (i, em, ep)
        assert np.isfinite(deltas[i])


def ct_batch():
    return wl.concat_tracks([wl.ct_bearings(T, seed=60 + T) for T in (40, 300, 7, 1, 120)], "ragged")


@pytest.mark.parametrize("lanes,slots,scan", [(64, 1, "parallel"), (64, 8, "parallel"), (256, 3, "parallel"),
                                              (0, 0, "sequential")])
@pytest.mark.parametrize("lin", ["taylor", "cubature"])
@pytest.mark.parametrize("bad", [0, 1, 4])
def test_ct_batch(B, lanes, slots, scan, lin, bad):
    pb = ct_batch()
    out = run_with_failed_track(B, pb, bad, lin, tile_lanes=lanes, lane_slots=slots, scan=scan)
    check_others(pb, bad, lin, *out, tol=1e-9)


def test_fp32(B):
    pb = ct_batch()
    out = run_with_failed_track(B, pb, 1, "taylor", precision="f32")
    check_others(pb, 1, "taylor", *out, tol=1e-4)


@pytest.mark.parametrize("slots", [1, 8])
@pytest.mark.parametrize("bad", [0, 1])
def test_dense_stacked_batch(B, slots, bad):
    sensors = np.random.default_rng([5, 0]).uniform(-2.0, 2.0, (8, 2))
    parts = [wl.stacked_ct(T, np.random.default_rng([57, T]), sensors=sensors) for T in (30, 9, 70)]
    pb = wl.concat_tracks(parts, "stacked batch")
    out = run_with_failed_track(B, pb, bad, "unscented", lane_slots=slots)
    check_others(pb, bad, "unscented", *out, tol=1e-9)


@pytest.mark.parametrize("lanes,slots", [(64, 1), (256, 3)])
def test_iterate_until_runs_the_other_tracks_on(B, lanes, slots):
    """smoother_iterate_until with a failed track: the others converge at the
    iterations they take without it, with the same results bit for bit, and
    the call reports the failure."""
    import torch
    pb = ct_batch()
    L = pb.lengths
    so = pb.slot_offsets()
    bad = 1
    clean = torch.from_numpy(np.repeat(pb.m0, L + 1, axis=0)).to("cuda", torch.float64)
    cov = torch.from_numpy(np.repeat(pb.P0, L + 1, axis=0)).to("cuda", torch.float64)
    broken = clean.clone()
    broken[so[bad] + 5, 2] = float("inf")
    torch.cuda.synchronize()
    kw = dict(n_iter=1, tile_lanes=lanes, lane_slots=slots)
    with B.Smoother(pb, **kw) as a, B.Smoother(pb, **kw) as b, B.Smoother(pb, **kw) as c:
        a.set_trajectory_device(broken.data_ptr(), cov.data_ptr())
        b.set_trajectory_device(clean.data_ptr(), cov.data_ptr())
        c.set_trajectory_device(clean.data_ptr(), cov.data_ptr())
        run_a, first_a, ok_a = a.iterate_until(1e-8, 40)
        run_b, first_b, ok_b = b.iterate_until(1e-8, 40)
        c.iterate(run_a)
        ma, ca = a.result()
        mc, cc = c.result()
    print(f"failed track {bad}: runs {run_a} / {run_b}, first {list(first_a)} / {list(first_b)}", flush=True)
    assert ok_b and not ok_a
    assert first_a[bad] == 0 and first_b[bad] > 0
    others = [i for i in range(pb.n_tracks) if i != bad]
    assert all(first_a[i] == first_b[i] > 0 for i in others), (first_a, first_b)
    assert run_a == max(first_a[i] for i in others)
    for i in others:
        sl = slice(so[i], so[i + 1])
        assert np.array_equal(ma[sl], mc[sl]) and np.array_equal(ca[sl], cc[sl]), i


def test_iterate_lm_runs_the_other_tracks_on(B):
    """smoother_iterate_lm with a failed track (objective not finite from the
    start): the others take the passes they take without it, and the failed
    track shows as a non-finite objective."""
    import torch
    pb = ct_batch()
    L = pb.lengths
    so = pb.slot_offsets()
    bad = 2
    clean = torch.from_numpy(np.repeat(pb.m0, L + 1, axis=0)).to("cuda", torch.float64)
    cov = torch.from_numpy(np.repeat(pb.P0, L + 1, axis=0)).to("cuda", torch.float64)
    broken = clean.clone()
    broken[so[bad] + 3, 1] = float("nan")
    torch.cuda.synchronize()
    with B.Smoother(pb, n_iter=1, tile_lanes=64, lane_slots=2) as a, \
            B.Smoother(pb, n_iter=1, tile_lanes=64, lane_slots=2) as b:
        a.set_trajectory_device(broken.data_ptr(), cov.data_ptr())
        b.set_trajectory_device(clean.data_ptr(), cov.data_ptr())
        run_a, first_a, cost_a = a.iterate_lm(tol=1e-8, max_iter=40)
        run_b, first_b, cost_b = b.iterate_lm(tol=1e-8, max_iter=40)
    print(f"LM, failed track {bad}: passes {run_a} / {run_b}, first {list(first_a)} / {list(first_b)}", flush=True)
    assert first_a[bad] == 0 and not np.isfinite(cost_a[bad])
    others = [i for i in range(pb.n_tracks) if i != bad]
    assert all(first_a[i] == first_b[i] > 0 for i in others), (first_a, first_b)
    assert run_a == max(first_a[i] for i in others)
    assert np.all(np.isfinite(cost_a[others]))
    if run_a == run_b:
        assert np.array_equal(cost_a[others], cost_b[others])
