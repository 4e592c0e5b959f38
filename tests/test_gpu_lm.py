"""GPU parity of Levenberg-Marquardt damped iterations (Section 3, the damped
Gauss-Newton extension of the iterated smoother) against the oracle's damped
smoother, on every engine: the nx = 5 scan kernels (Taylor and sigma points,
FP64 and FP32, parallel and sequential), the linear models, stacked Taylor
targets (per-target blocks) and the nx = 20 wavefront-cooperative engine.

Metric and FP64 gate as in test_gpu_parity.  The damping observes the previous
iterate at every slot, so a one-iteration comparison from a common input
trajectory checks the damped element build directly.
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
        sm.iterate(0)
        mean, cov = sm.result()
        deltas = sm.track_deltas()
    return mean, cov, deltas


def assert_parity(mean, cov, ref, tol=TOL64, what=""):
    em = oracle.mean_error(mean, ref["mean"])
    ep = oracle.cov_error(cov, ref["cov"])
    print(f"{what}: e_m={em:.3e} e_P={ep:.3e}", flush=True)
    assert em < tol and ep < tol, (what, em, ep)


def one_iteration(B, pb, lin, start, lam, **kw):
    """Damped iteration start+1 on the GPU from the oracle's damped iterate `start`."""
    ref = oracle.smoother(pb, start + 1, lin, history=True, lm_lambda=lam)
    im = None if start == 0 else ref["hist_mean"][start - 1]
    ic = None if start == 0 else ref["hist_cov"][start - 1]
    mean, cov, _ = run_gpu(B, pb, 1, lin, init_mean=im, init_cov=ic, lm_lambda=lam, **kw)
    return mean, cov, {"mean": ref["hist_mean"][start], "cov": ref["hist_cov"][start]}


@pytest.mark.parametrize("lin", ["taylor", "cubature", "unscented"])
@pytest.mark.parametrize("lam", [0.05, 2.0])
def test_c1_damped_iterations(B, lin, lam):
    pb = wl.config_c1()
    for start in (0, 3):
        mean, cov, one = one_iteration(B, pb, lin, start, lam)
        assert_parity(mean, cov, one, what=f"C1 {lin} lambda={lam} iteration {start + 1}")


def test_c1_ten_damped_iterations(B):
    pb = wl.config_c1()
    ref = oracle.smoother(pb, 10, "taylor", lm_lambda=0.5)
    mean, cov, deltas = run_gpu(B, pb, 10, "taylor", lm_lambda=0.5)
    assert abs(deltas[0] - ref["deltas"][-1]) <= 1e-6 * ref["deltas"][-1] + 1e-12
    assert_parity(mean, cov, ref, what="C1 taylor lambda=0.5 M=10")


@pytest.mark.parametrize("T", [1, 2, 65, 513, 32768])
def test_tile_edges_and_c2_size(B, T):
    pb = wl.config_c2(T) if T > 1 else wl.ct_bearings(1, seed=5)
    for start in (0, 2):
        mean, cov, one = one_iteration(B, pb, "taylor", start, 0.3)
        assert_parity(mean, cov, one, what=f"T={T} lambda=0.3 iteration {start + 1}")


@pytest.mark.parametrize("lanes,slots", [(64, 3), (256, 8)])
def test_schedules(B, lanes, slots):
    pb = wl.config_c2(3000)
    mean, cov, one = one_iteration(B, pb, "cubature", 1, 1.0, tile_lanes=lanes, lane_slots=slots)
    assert_parity(mean, cov, one, what=f"{lanes}x{slots} cubature lambda=1")


def test_sequential_mode(B):
    pb = wl.config_c1()
    for lin in ("taylor", "cubature"):
        mean, cov, one = one_iteration(B, pb, lin, 2, 0.5, scan="sequential")
        assert_parity(mean, cov, one, what=f"sequential C1 {lin} lambda=0.5")


def test_ragged_batch(B):
    """Damping of every track's prior element and of its interior slots."""
    pb = wl.concat_tracks([wl.ct_bearings(1, seed=1), wl.ct_bearings(70, seed=2), wl.ct_bearings(300, seed=3),
                           wl.ct_bearings(2, seed=4)], "ragged")
    M, lam = 3, 0.7
    mean, cov, deltas = run_gpu(B, pb, M, "taylor", lm_lambda=lam)
    so = pb.slot_offsets()
    for i in range(pb.n_tracks):
        ref = oracle.smoother(pb.track(i), M, "taylor", lm_lambda=lam)
        sl = slice(so[i], so[i + 1])
        assert_parity(mean[sl], cov[sl], ref, what=f"track {i} T={pb.lengths[i]}")
        assert abs(deltas[i] - ref["deltas"][-1]) <= 1e-6 * ref["deltas"][-1] + 1e-12


@pytest.mark.parametrize("nx,ny,T", [(1, 1, 700), (3, 2, 1000)])
def test_linear_models(B, nx, ny, T):
    pb = wl.linear_gaussian(nx, ny, T, seed=7)
    ref = oracle.smoother(pb, 2, "taylor", lm_lambda=0.4)
    mean, cov, _ = run_gpu(B, pb, 2, "taylor", lm_lambda=0.4)
    assert_parity(mean, cov, ref, what=f"linear({nx},{ny}) lambda=0.4")


def test_fp32(B):
    pb = wl.config_c1()
    ref = oracle.smoother(pb, 10, "taylor", lm_lambda=0.5)
    mean, cov, _ = run_gpu(B, pb, 10, "taylor", precision="f32", lm_lambda=0.5)
    em = oracle.mean_error(mean, ref["mean"])
    ep = oracle.cov_error(cov, ref["cov"])
    print(f"FP32 C1 lambda=0.5: e_m={em:.3e} e_P={ep:.3e}", flush=True)
    assert em < 1e-4 and ep < 1e-4


def _block_diag_only(c, k=4):
    out = np.zeros_like(c)
    for b in range(k):
        sl = slice(5 * b, 5 * b + 5)
        out[..., sl, sl] = c[..., sl, sl]
    return out


def test_stacked_taylor_blocks(B):
    pb = wl.config_c5_single(300)
    lam = 0.5
    ref = oracle.smoother(pb, 2, "taylor", history=True, lm_lambda=lam)
    for start in (0, 1):
        im = None if start == 0 else ref["hist_mean"][start - 1]
        ic = None if start == 0 else _block_diag_only(ref["hist_cov"][start - 1])
        one = {"mean": ref["hist_mean"][start], "cov": ref["hist_cov"][start]}
        mean, cov, _ = run_gpu(B, pb, 1, "taylor", init_mean=im, init_cov=ic, lm_lambda=lam)
        assert_parity(mean, cov, one, what=f"stacked n=20 taylor lambda={lam} iteration {start + 1}")


@pytest.mark.parametrize("slots", [1, 8])
def test_dense_sigma_points(B, slots):
    pb = wl.config_c5_single(300)
    for start in (0, 2):
        mean, cov, one = one_iteration(B, pb, "unscented", start, 0.5, lane_slots=slots)
        assert_parity(mean, cov, one, what=f"dense n=20 unscented lambda=0.5 slots={slots} iteration {start + 1}")


@pytest.mark.parametrize("precision,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_dense_damped_kernel_at_vanishing_lambda(B, precision, tol):
    """The n = 20 engine launches a level-0 filtering kernel with a larger LDS
    work area when lambda > 0 (the damping's scratch) and the seven-matrix one
    otherwise.  At lambda = 1e-300 the damping changes nothing measurable, so
    the two kernels must agree on a ragged batch over two iterations."""
    pb = wl.config_c5_batch(6, 200, 700)
    kw = dict(lane_slots=4, precision=precision)
    m0, c0, _ = run_gpu(B, pb, 2, "unscented", **kw)
    m1, c1, _ = run_gpu(B, pb, 2, "unscented", lm_lambda=1e-300, **kw)
    em = float(np.max(np.abs(m1 - m0)) / max(1.0, float(np.max(np.abs(m0)))))
    ep = float(np.max(np.abs(c1 - c0)) / max(1.0, float(np.max(np.abs(c0)))))
    print(f"damped vs undamped kernel, lambda=1e-300, {precision}: {em:.2e} {ep:.2e}", flush=True)
    assert np.all(np.isfinite(m0)) and np.all(np.isfinite(c0))
    assert em < tol and ep < tol, (em, ep)


def test_damped_fixed_point_is_undamped_fixed_point(B):
    """Section 3: the damping term vanishes at a fixed point, so damped and
    undamped iterations converge to the same trajectory."""
    pb = wl.config_c1()
    plain, _, _ = run_gpu(B, pb, 40, "taylor")
    damped, _, _ = run_gpu(B, pb, 120, "taylor", lm_lambda=0.1)
    err = oracle.mean_error(damped, plain)
    print(f"damped vs plain fixed point: {err:.3e}", flush=True)
    assert err < 1e-8


# ---------------------------------------------------------------------------------------
# MAP objective and Levenberg-Marquardt with Marquardt's damping schedule.
# ---------------------------------------------------------------------------------------
def _perturbed_batch_init(pb, scale, seed):
    rng = np.random.default_rng(seed)
    so = pb.slot_offsets()
    im = np.concatenate([np.broadcast_to(pb.m0[i], (so[i + 1] - so[i], pb.nx)) for i in range(pb.n_tracks)])
    return im + scale * rng.standard_normal(im.shape)


@pytest.mark.parametrize("kind", ["ct", "linear", "stacked"])
def test_objective_matches_oracle(B, kind):
    if kind == "ct":
        pb = wl.concat_tracks([wl.ct_bearings(T, seed=T) for T in (1, 2, 63, 700)], "ragged")
    elif kind == "linear":
        pb = wl.linear_gaussian(3, 2, 300, seed=4, n_tracks=3, t_min=1)
    else:
        sensors = np.random.default_rng([5, 0]).uniform(-2.0, 2.0, (8, 2))
        pb = wl.concat_tracks([wl.stacked_ct(T, np.random.default_rng([57, T]), sensors=sensors)
                               for T in (3, 120)], "stacked batch")
    im = _perturbed_batch_init(pb, 0.3, 1)
    with B.Smoother(pb, n_iter=1, init_mean=im) as sm:
        got = sm.objective()
    so = pb.slot_offsets()
    for i in range(pb.n_tracks):
        ref = oracle.map_cost(pb.track(i), im[so[i]:so[i + 1]])
        print(f"{kind} track {i}: {got[i]:.15e} vs {ref:.15e}", flush=True)
        assert abs(got[i] - ref) <= 1e-12 * abs(ref)


def test_objective_fp32(B):
    pb = wl.config_c1()
    im = _perturbed_batch_init(pb, 0.3, 2)
    with B.Smoother(pb, n_iter=1, init_mean=im, precision="f32") as sm:
        got = sm.objective()[0]
    ref = oracle.map_cost(pb, im)
    assert abs(got - ref) <= 1e-5 * abs(ref)


def _margins_clear(ref, J0, rtol=1e-12):
    """The oracle's keep/reject decisions are not within rounding of the threshold."""
    prev = np.concatenate([[J0], ref["cost"][:-1]])
    m = ref["cost_new"] - (prev + rtol * np.abs(prev))
    return np.all(np.abs(m) > 1e-14 * np.abs(prev))


def test_adaptive_single_track_matches_oracle(B):
    pb = wl.config_c1()
    with B.Smoother(pb, n_iter=1) as sm:
        run, first, cost = sm.iterate_lm(1e-2, 10.0, 1e-9, 200)
        mean, cov = sm.result()
    ref = oracle.lm_adaptive(pb, 1e-2, 10.0, 1e-9, 200)
    J0 = oracle.map_cost(pb, np.broadcast_to(pb.m0[0], mean.shape))
    assert _margins_clear(ref, J0)
    print(f"C1 adaptive: gpu run={run} first={first[0]}, oracle {ref['iters']} {ref['first']}", flush=True)
    assert run == ref["iters"] and first[0] == ref["first"] > 0
    assert abs(cost[0] - ref["final_cost"]) <= 1e-12 * ref["final_cost"]
    assert_parity(mean, cov, ref, what="C1 adaptive damping")


def test_adaptive_batch_matches_oracle(B):
    """Held-out warm-start tracks (T = 4096): two where undamped iterations do
    not converge in 100 passes (145, 147), one slow (38) and two ordinary."""
    idx = (0, 38, 145, 147, 3)
    pb = wl.concat_tracks([wl.config_c4(i, 1, held_out=True) for i in idx], "held-out")
    with B.Smoother(pb, n_iter=1) as sm:
        run, first, cost = sm.iterate_lm(1e-2, 10.0, 1e-6, 80)
        mean, cov = sm.result()
    so = pb.slot_offsets()
    assert np.all(first > 0)
    for i in range(pb.n_tracks):
        tr = pb.track(i)
        ref = oracle.lm_adaptive(tr, 1e-2, 10.0, 1e-6, run, stop=False)
        J0 = oracle.map_cost(tr, np.broadcast_to(tr.m0[0], (so[i + 1] - so[i], 5)))
        assert _margins_clear(ref, J0), i
        print(f"track {idx[i]}: first gpu {first[i]} oracle {ref['first']}", flush=True)
        assert first[i] == ref["first"]
        assert abs(cost[i] - ref["final_cost"]) <= 1e-10 * ref["final_cost"]
        sl = slice(so[i], so[i + 1])
        assert_parity(mean[sl], cov[sl], ref, tol=1e-8, what=f"held-out track {idx[i]} adaptive")


def test_adaptive_batch_with_lane_runs(B):
    """The damping schedule with several slots per lane (restore by column)."""
    idx = (145, 3, 38)
    pb = wl.concat_tracks([wl.config_c4(i, 1, held_out=True) for i in idx], "held-out")
    with B.Smoother(pb, n_iter=1, tile_lanes=64, lane_slots=8) as sm:
        run, first, cost = sm.iterate_lm(1e-2, 10.0, 1e-6, 60)
        mean, cov = sm.result()
    so = pb.slot_offsets()
    for i in range(pb.n_tracks):
        tr = pb.track(i)
        ref = oracle.lm_adaptive(tr, 1e-2, 10.0, 1e-6, run, stop=False)
        print(f"64x8 track {idx[i]}: first gpu {first[i]} oracle {ref['first']}", flush=True)
        assert first[i] == ref["first"] > 0
        sl = slice(so[i], so[i + 1])
        assert_parity(mean[sl], cov[sl], ref, tol=1e-8, what=f"64x8 adaptive track {idx[i]}")


def test_adaptive_stacked_blocks_match_dense_oracle(B):
    pb = wl.config_c5_single(200)
    with B.Smoother(pb, n_iter=1) as sm:
        run, first, cost = sm.iterate_lm(1e-2, 10.0, 1e-9, 100)
        mean, cov = sm.result()
    ref = oracle.lm_adaptive(pb, 1e-2, 10.0, 1e-9, 100)
    print(f"stacked adaptive: gpu run={run} first={first[0]}, oracle {ref['iters']} {ref['first']}", flush=True)
    assert run == ref["iters"] and first[0] == ref["first"] > 0
    assert_parity(mean, _block_diag_only(cov), {"mean": ref["mean"], "cov": _block_diag_only(ref["cov"])},
                  tol=1e-8, what="stacked adaptive")


def test_adaptive_modes_agree_and_plain_pass_follows(B):
    """Graph replay, eager launches and the sequential path take the same
    passes; afterwards smoother_iterate runs undamped again."""
    pb = wl.config_c1()
    outs = []
    for kw in ({}, {"use_graph": False}, {"scan": "sequential"}):
        with B.Smoother(pb, n_iter=1, **kw) as sm:
            run, first, _ = sm.iterate_lm(1e-2, 10.0, 1e-8, 100)
            m, c = sm.result()
            sm.iterate(1)
            m2, c2 = sm.result()
        outs.append((run, first[0], m, c, m2, c2))
    assert outs[0][:2] == outs[1][:2] == outs[2][:2]
    assert np.array_equal(outs[0][2], outs[1][2]) and np.array_equal(outs[0][4], outs[1][4])
    assert oracle.mean_error(outs[2][2], outs[0][2]) < 1e-10
    ref = oracle.smoother(pb, 1, "taylor", init_mean=outs[0][2], init_cov=outs[0][3])
    assert_parity(outs[0][4], outs[0][5], ref, what="undamped pass after adaptive damping")


def test_adaptive_fp32(B):
    pb = wl.config_c1()
    with B.Smoother(pb, n_iter=1, precision="f32") as sm:
        run, first, _ = sm.iterate_lm(1e-2, 10.0, 1e-4, 100)
        mean, _ = sm.result()
    ref = oracle.lm_adaptive(pb, 1e-2, 10.0, 1e-9, 200)
    err = oracle.mean_error(mean, ref["mean"])
    print(f"FP32 adaptive: run={run} first={first[0]} e_m={err:.3e}", flush=True)
    assert first[0] > 0 and err < 1e-4


def test_adaptive_needs_taylor_and_objective_engine(B):
    with B.Smoother(wl.config_c1(), n_iter=1, lin="cubature") as sm:
        with pytest.raises(B.SmootherError, match="Taylor"):
            sm.iterate_lm()
    with B.Smoother(wl.config_c5_single(20), n_iter=1, lin="unscented") as sm:
        with pytest.raises(B.SmootherError, match="not built"):
            sm.iterate_lm()


def _c5_batch_track(i):
    """Track i of the C5 batch on its own: its length, states and noises come
    from default_rng([5, 1 + i]) in the batch's order (stacked_ct draws the
    same; only the rounding of the noise products may differ)."""
    rng = np.random.default_rng([5, 1 + i])
    T = int(rng.integers(1024, 2 ** 16 + 1))
    sensors = np.random.default_rng([5, 0]).uniform(-2.0, 2.0, (8, 2))
    return wl.stacked_ct(T, rng, sensors=sensors)


def test_damping_holds_a_diverging_stacked_track(B):
    """C5 batch track 180 (T = 62736, four targets, unscented) diverges under
    the undamped iteration: its means pass 1e4 within two iterations.  With a
    fixed damping lambda = 10 (Section 3's damped extension) the iterates stay
    bounded, and the device's third damped iterate equals the oracle's."""
    pb = _c5_batch_track(180)
    assert pb.lengths[0] == 62736
    mean, _, _ = run_gpu(B, pb, 2, "unscented")
    undamped = float(np.nanmax(np.abs(mean)))
    M, lam = 3, 10.0
    ref = oracle.smoother(pb, M, "unscented", lm_lambda=lam, filtered=False)
    mean, cov, deltas = run_gpu(B, pb, M, "unscented", lm_lambda=lam)
    damped = float(np.max(np.abs(mean)))
    print(f"track 180: max |mean| undamped after 2 iterations {undamped:.3e}, damped (lambda={lam}) after {M} "
          f"{damped:.3e}", flush=True)
    assert undamped > 1e4 and damped < 100.0
    assert_parity(mean, cov, ref, what=f"track 180 damped lambda={lam} M={M}")
    assert abs(deltas[0] - ref["deltas"][-1]) <= 1e-6 * ref["deltas"][-1] + 1e-12
