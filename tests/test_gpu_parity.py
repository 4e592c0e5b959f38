"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Metric (per slot, worst slot reported):
  e_m = ||m_gpu - m_or||_2 / max(||m_or||_2, 1e-3),  e_P = ||P_gpu - P_or||_F / ||P_or||_F.
FP64 gate 1e-9.  Multi-iteration comparisons are made where the iterated
smoother converges; elsewhere each iteration is compared from a common input
trajectory (the oracle's previous iterate), which removes the amplification
of rounding differences by a not-yet-converged Gauss-Newton / posterior
linearisation iteration.
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


def run_gpu(B, pb, M, lin="taylor", **kw):
    with B.Smoother(pb, n_iter=M, lin=lin, **kw) as sm:
        delta, iters = sm.iterate(0)
        mean, cov = sm.result()
        deltas = sm.track_deltas()
    return mean, cov, delta, deltas


def assert_parity(mean, cov, ref, tol=TOL64, what=""):
    em = oracle.mean_error(mean, ref["mean"])
    ep = oracle.cov_error(cov, ref["cov"])
    print(f"{what}: e_m={em:.3e} e_P={ep:.3e}", flush=True)
    assert em < tol and ep < tol, (what, em, ep)


@pytest.mark.parametrize("lin", ["taylor", "cubature", "unscented"])
def test_c1_ten_iterations(B, lin):
    pb = wl.config_c1()
    ref = oracle.smoother(pb, 10, lin)
    mean, cov, delta, _ = run_gpu(B, pb, 10, lin)
    assert abs(delta - ref["deltas"][-1]) <= 1e-6 * max(ref["deltas"][-1], 1e-12) + 1e-12
    assert_parity(mean, cov, ref, what=f"C1 {lin} M=10")


@pytest.mark.parametrize("nx,ny,T,seed", [(1, 1, 700, 3), (3, 2, 1000, 1), (5, 2, 257, 2)])
@pytest.mark.parametrize("lin", ["taylor", "cubature"])
def test_linear_models(B, nx, ny, T, seed, lin):
    pb = wl.linear_gaussian(nx, ny, T, seed=seed)
    ref = oracle.smoother(pb, 2, lin)
    mean, cov, _, _ = run_gpu(B, pb, 2, lin)
    assert_parity(mean, cov, ref, what=f"linear({nx},{ny}) T={T} {lin}")


@pytest.mark.parametrize("T", [1, 2, 3, 63, 64, 65, 127, 128, 129, 511, 512, 513, 1000])
def test_tile_edges(B, T):
    """Lengths around the lane (K), tile (64 lanes) and top-level boundaries."""
    pb = wl.config_c2(T) if T > 1 else wl.ct_bearings(1, seed=5)
    ref = oracle.smoother(pb, 3, "taylor")
    mean, cov, _, _ = run_gpu(B, pb, 3)
    assert_parity(mean, cov, ref, what=f"T={T}")


def single_iteration_case(B, pb, lin, start_iter):
    """Compare iteration start_iter+1 from the oracle's iterate start_iter."""
    ref = oracle.smoother(pb, start_iter + 1, lin, history=True)
    if start_iter == 0:
        im, ic = None, None
    else:
        im, ic = ref["hist_mean"][start_iter - 1], ref["hist_cov"][start_iter - 1]
    one = {"mean": ref["hist_mean"][start_iter], "cov": ref["hist_cov"][start_iter]}
    mean, cov, _, _ = run_gpu(B, pb, 1, lin, init_mean=im, init_cov=ic)
    return mean, cov, one


@pytest.mark.parametrize("T", [1024, 4096, 32768])
@pytest.mark.parametrize("lin", ["taylor", "cubature"])
def test_c2_single_iteration(B, T, lin):
    pb = wl.config_c2(T)
    for start in (0, 4):
        mean, cov, one = single_iteration_case(B, pb, lin, start)
        assert_parity(mean, cov, one, what=f"C2 T={T} {lin} iteration {start + 1}")


def test_long_tracks(B):
    """Long single tracks (automatic schedule)."""
    pb = wl.ct_bearings(20000, seed=7)
    mean, cov, one = single_iteration_case(B, pb, "taylor", 0)
    assert_parity(mean, cov, one, what="T=20000")
    p2 = wl.linear_gaussian(1, 1, 70000, seed=4)
    ref = oracle.smoother(p2, 1, "taylor")
    mean, cov, _, _ = run_gpu(B, p2, 1)
    assert_parity(mean, cov, ref, what="linear T=70000")


def test_sequential_mode_matches_oracle(B):
    pb = wl.config_c1()
    ref = oracle.smoother(pb, 10, "cubature")
    mean, cov, _, _ = run_gpu(B, pb, 10, "cubature", scan="sequential")
    assert_parity(mean, cov, ref, what="sequential C1 cubature")


def test_ragged_batch_equals_single_tracks(B):
    pb = wl.ct_batch(24, 1, 300, seed_tag=11)
    pb = wl.concat_tracks([wl.ct_bearings(1, seed=1), wl.ct_bearings(2, seed=2), pb.track(0), pb,
                           wl.ct_bearings(1, seed=3)], "ragged")
    M = 4
    mean, cov, _, deltas = run_gpu(B, pb, M, "cubature")
    so = pb.slot_offsets()
    for i in range(pb.n_tracks):
        ref = oracle.smoother(pb.track(i), M, "cubature")
        sl = slice(so[i], so[i + 1])
        assert_parity(mean[sl], cov[sl], ref, what=f"track {i} T={pb.lengths[i]}")
        assert abs(deltas[i] - ref["deltas"][-1]) <= 1e-6 * ref["deltas"][-1] + 1e-12


def test_deterministic(B):
    pb = wl.config_c2(4096)
    a = run_gpu(B, pb, 3, "cubature")
    b = run_gpu(B, pb, 3, "cubature")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_resume_is_bitwise(B):
    pb = wl.config_c2(2048)
    full = run_gpu(B, pb, 6)
    half = run_gpu(B, pb, 3)
    rest = run_gpu(B, pb, 3, init_mean=half[0], init_cov=half[1])
    assert np.array_equal(full[0], rest[0]) and np.array_equal(full[1], rest[1])


def test_result_device_into_torch(B):
    import torch
    pb = wl.config_c1()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with B.Smoother(pb, stream=stream.cuda_stream, n_iter=10) as sm:
            sm.iterate(0, want_delta=False)
            S, _, _ = sm.info()
            m = torch.empty((S, 5), dtype=torch.float64, device="cuda")
            P = torch.empty((S, 5, 5), dtype=torch.float64, device="cuda")
            sm.result_device(m.data_ptr(), P.data_ptr())
            hm, hP = sm.result()
    stream.synchronize()
    assert np.array_equal(m.cpu().numpy(), hm) and np.array_equal(P.cpu().numpy(), hP)


def test_fp32_variant(B):
    pb = wl.config_c1()
    ref = oracle.smoother(pb, 10, "taylor")
    mean, cov, _, _ = run_gpu(B, pb, 10, "taylor", precision="f32")
    em = oracle.mean_error(mean, ref["mean"])
    ep = oracle.cov_error(cov, ref["cov"])
    print(f"FP32 C1: e_m={em:.3e} e_P={ep:.3e}", flush=True)
    assert em < 1e-4 and ep < 1e-3


@pytest.mark.parametrize("lanes,slots", [(64, 1), (64, 2), (64, 3), (256, 1), (256, 2), (256, 4), (256, 8)])
@pytest.mark.parametrize("T", [1, 5, 200, 3000])
def test_schedules(B, lanes, slots, T):
    """Every (lanes per tile, slots per lane) gives the oracle's result,
    including partially filled and padded tiles."""
    pb = wl.config_c2(T) if T > 1 else wl.ct_bearings(1, seed=5)
    ref = oracle.smoother(pb, 2, "cubature")
    mean, cov, _, _ = run_gpu(B, pb, 2, "cubature", tile_lanes=lanes, lane_slots=slots)
    assert_parity(mean, cov, ref, what=f"T={T} lanes={lanes} slots={slots}")


def test_multilevel_tile_scan(B):
    """More tile aggregates than one block scans: the generic multi-level scan
    runs between the fused kernels (64 lanes x 1 slot -> 1094 tiles)."""
    p2 = wl.linear_gaussian(1, 1, 70000, seed=4)
    ref = oracle.smoother(p2, 1, "taylor")
    with B.Smoother(p2, n_iter=1, tile_lanes=64, lane_slots=1) as sm:
        lanes, slots, tiles = sm.schedule()
        assert tiles > 64 * 8
        sm.iterate(0)
        mean, cov = sm.result()
    assert_parity(mean, cov, ref, what="linear T=70000, 1094 tiles")


@pytest.mark.parametrize("lin", ["taylor", "cubature"])
def test_graph_replays_match_eager(B, lin):
    """Each iteration replayed from the captured HIP graph equals the same
    iteration launched kernel by kernel, replay after replay, with other
    eager work and host synchronisation in between."""
    import torch
    pb = wl.concat_tracks([wl.config_c2(3000), wl.ct_bearings(1, seed=4), wl.ct_batch(6, 20, 500, seed_tag=13)])
    g = B.Smoother(pb, n_iter=6, lin=lin, use_graph=True)
    e = B.Smoother(pb, n_iter=6, lin=lin, use_graph=False)
    scratch = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
    try:
        for i in range(5):
            dg, _ = g.iterate(1)
            scratch.mul_(1.0000001)               # unrelated eager work on the device
            de, _ = e.iterate(1)
            torch.cuda.synchronize()
            mg, Pg = g.result()
            me, Pe = e.result()
            assert dg == de and np.array_equal(mg, me) and np.array_equal(Pg, Pe), i
    finally:
        g.close()
        e.close()
