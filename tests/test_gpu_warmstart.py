"""GPU checks of the learned initial trajectory: the network's kernels (forward,
gradient, Adam, window / label / trajectory layouts) against the FP64 NumPy
oracle of the same network, the device-trajectory entry point of the smoother
against its host-input path, and a small end-to-end run that trains the
network on smoother outputs and shows what it gains over the prior start.

FP32 tolerances: a forward value is a sum of at most C * 3 = 384 products per
layer over 6 layers, so its error is a few hundred FP32 ulps of the activation
scale at worst (bound 1e-5 relative to the largest output used); a gradient
entry sums up to n * L = 16384 products (bound 2e-4 of the layer's gradient
norm)."""
import numpy as np
import pytest

from oracle import nn as onn
from paper_2102_00514_amd import workloads as wl

pytestmark = pytest.mark.gpu

SMALL = dict(window=16, patch=4, width=16, hidden=2, nx=5, ny=2)


@pytest.fixture(scope="module")
def W():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2102_00514_amd import warmstart
    return warmstart


def _net(W, cfgd, max_batch, seed=0):
    import torch
    cfg = W.config(max_batch=max_batch, **cfgd)
    return W.WarmStartNet(cfg, stream=torch.cuda.current_stream().cuda_stream, seed=seed)


def _data(cfgd, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, 2 * cfgd["ny"], cfgd["window"])).astype(np.float32)
    lab = rng.standard_normal((n, cfgd["window"], cfgd["nx"])).astype(np.float32) * 2 + 0.5
    return x, lab


def _dev(a):
    """Device copy; the caller keeps the tensor referenced while kernels use its pointer."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("cfgd,n,max_batch", [(SMALL, 7, 8), (SMALL, 20, 8), (onn.DEFAULT, 40, 64)])
def test_forward_matches_oracle(W, cfgd, n, max_batch):
    import torch
    net = _net(W, cfgd, max_batch, seed=3)
    mu = np.array([0.3, -0.2, 1.0, 0.0, 0.1], np.float32)
    sigma = np.array([2.0, 1.5, 0.7, 0.7, 0.4], np.float32)
    net.set_normalization(mu, sigma)
    x, _ = _data(cfgd, n, 1)
    idx = np.random.default_rng(2).permutation(n).astype(np.int32)
    out = torch.empty((n, cfgd["window"], 5), dtype=torch.float32, device="cuda")
    dx, didx = _dev(x), _dev(idx)          # kept alive until the kernels have read them
    net.predict(dx.data_ptr(), n, didx.data_ptr(), n, out.data_ptr())
    ref_o, _ = onn.forward(net.params().astype(np.float64), x[idx].astype(np.float64), cfgd)
    ref = onn.outputs_to_states(ref_o, mu.astype(np.float64), sigma.astype(np.float64), cfgd)
    got = out.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"forward {cfgd['width']}x{cfgd['hidden']} n={n}: rel err {err:.2e}", flush=True)
    assert err < 1e-5
    net.close()


def _layer_slices(cfgd):
    pos, out = 0, []
    for ws, bs in onn.layer_shapes(cfgd):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append(slice(pos, pos + nw))
        out.append(slice(pos + nw, pos + nw + nb))
        pos += nw + nb
    return out


@pytest.mark.parametrize("cfgd,n,max_batch", [(SMALL, 6, 6), (onn.DEFAULT, 48, 64), (dict(onn.DEFAULT, hidden=0), 9, 16)])
def test_gradient_matches_oracle(W, cfgd, n, max_batch):
    net = _net(W, cfgd, max_batch, seed=4)
    # trained-looking parameters: non-zero biases and head so every path carries gradient
    rng = np.random.default_rng(5)
    theta = net.params().astype(np.float64)
    theta += 0.05 * rng.standard_normal(theta.size)
    net.set_params(theta.astype(np.float32))
    theta = net.params().astype(np.float64)
    mu = np.array([0.5, 0.0, 0.2, -0.1, 0.0], np.float32)
    sigma = np.array([1.5, 1.0, 0.8, 0.9, 0.5], np.float32)
    net.set_normalization(mu, sigma)
    x, lab = _data(cfgd, 3 * n, 6)
    idx = rng.choice(3 * n, size=n, replace=False).astype(np.int32)
    dx, dl, didx = _dev(x), _dev(lab), _dev(idx)
    g, loss = net.gradient(dx.data_ptr(), dl.data_ptr(), 3 * n, didx.data_ptr(), n)
    tgt = onn.states_to_outputs(lab[idx].astype(np.float64), mu.astype(np.float64), sigma.astype(np.float64), cfgd)
    out, cache = onn.forward(theta, x[idx].astype(np.float64), cfgd)
    ref_loss = onn.loss(out, tgt)
    ref = onn.backward(theta, cache, out, tgt, cfgd)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    for sl in _layer_slices(cfgd):
        a, b = g[sl].astype(np.float64), ref[sl]
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert err < 2e-4, (sl, err)
    print(f"gradient {cfgd['width']}x{cfgd['hidden']}: loss {loss:.6f} vs {ref_loss:.6f}", flush=True)
    net.close()


def test_adam_steps_match_oracle(W):
    cfgd = SMALL
    net = _net(W, cfgd, 16, seed=7)
    net.set_normalization(np.zeros(5, np.float32), np.ones(5, np.float32))
    x, lab = _data(cfgd, 16, 8)
    dx, dl = _dev(x), _dev(lab)
    idx = _dev(np.arange(16, dtype=np.int32))
    theta = net.params().astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    lr = 1e-2
    for t in (1, 2, 3):
        g, _ = net.gradient(dx.data_ptr(), dl.data_ptr(), 16, idx.data_ptr(), 16)
        net.train_step(dx.data_ptr(), dl.data_ptr(), 16, idx.data_ptr(), 16, lr)
        theta, m, v = onn.adam_step(theta, g.astype(np.float64), m, v, t, lr)
        got = net.params().astype(np.float64)
        assert np.max(np.abs(got - theta)) < 1e-5 * lr + 1e-6 * np.max(np.abs(theta)), t
    net.close()


def test_windows_labels_trajectory_match_oracle(W):
    import torch
    cfgd = onn.DEFAULT
    net = _net(W, cfgd, 4, seed=9)     # max_batch 4: the trajectory runs in several chunks
    mu = np.array([0.1, 0.2, 1.0, 0.0, 0.0], np.float32)
    sigma = np.array([1.0, 1.0, 0.5, 0.5, 0.3], np.float32)
    net.set_normalization(mu, sigma)
    lengths = np.array([200, 64, 7, 129, 1, 65])
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    rng = np.random.default_rng(10)
    y = rng.uniform(-np.pi, np.pi, (int(offsets[-1]), 2))
    S = int((lengths + 1).sum())
    mean = rng.standard_normal((S, 5))
    nw = net.set_tracks(offsets)
    assert nw == len(onn.window_table(offsets))
    dy = _dev(y)
    X = torch.empty((nw, 4, 64), dtype=torch.float32, device="cuda")
    LAB = torch.empty((nw, 64, 5), dtype=torch.float32, device="cuda")
    net.windows(dy.data_ptr(), X.data_ptr())
    dmean = _dev(mean)
    net.labels(dmean.data_ptr(), LAB.data_ptr())
    ref_x = onn.features(y, offsets)
    assert np.max(np.abs(X.cpu().numpy() - ref_x)) < 2e-7
    np.testing.assert_array_equal(LAB.cpu().numpy(), onn.window_labels(mean, offsets).astype(np.float32))
    traj = torch.full((S, 5), float("nan"), dtype=torch.float64, device="cuda")
    net.trajectory(dy.data_ptr(), traj.data_ptr())
    o, _ = onn.forward(net.params().astype(np.float64), X.cpu().numpy().astype(np.float64), cfgd)
    ref_t = onn.trajectory(onn.outputs_to_states(o, mu.astype(np.float64), sigma.astype(np.float64)), offsets)
    got = traj.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref_t)) < 1e-5 * np.max(np.abs(ref_t))
    net.close()


def test_out_of_range_batch_index_is_reported(W):
    """An index past the data set reads nothing and the waiting call reports it."""
    net = _net(W, SMALL, 8, seed=1)
    x, lab = _data(SMALL, 4, 12)
    bad = _dev(np.array([0, 1, 4, 2], dtype=np.int32))
    dx, dl = _dev(x), _dev(lab)
    with pytest.raises(W.WarmStartError) as ei:
        net.gradient(dx.data_ptr(), dl.data_ptr(), 4, bad.data_ptr(), 4)
    assert ei.value.status == W.WS_EINVAL
    good = _dev(np.array([0, 1, 3, 2], dtype=np.int32))
    g, loss = net.gradient(dx.data_ptr(), dl.data_ptr(), 4, good.data_ptr(), 4)
    assert np.isfinite(loss) and np.all(np.isfinite(g))
    net.close()


def test_set_trajectory_device_equals_host_init(W):
    """The device entry point starts the smoother exactly where the host-input
    path (init_mean / init_cov) does."""
    import torch
    from paper_2102_00514_amd import binding as B
    pb = wl.concat_tracks([wl.config_c2(700), wl.ct_bearings(1, seed=3), wl.ct_batch(3, 50, 300, seed_tag=21)])
    S = pb.n_slots
    rng = np.random.default_rng(11)
    m_init = pb.truth + 0.1 * rng.standard_normal(pb.truth.shape)
    cconst = wl.random_spd(rng, 5, scale=0.2)
    dm = _dev(m_init)
    for lin in ("taylor", "cubature"):
        for cov_mode in ("const", "prior"):
            init_cov = np.broadcast_to(cconst, (S, 5, 5)) if cov_mode == "const" else None
            with B.Smoother(pb, n_iter=3, lin=lin, init_mean=m_init, init_cov=init_cov) as ref:
                ref.iterate(3)
                rm, rc = ref.result()
            with B.Smoother(pb, n_iter=3, lin=lin) as sm:
                sm.iterate(2)                       # state that the call must replace
                sm.set_trajectory_device(dm.data_ptr(), 0, cconst if cov_mode == "const" else None)
                d, it = sm.iterate(0)
                assert it == 3
                gm, gc = sm.result()
            assert np.array_equal(gm, rm) and np.array_equal(gc, rc), (lin, cov_mode)


def test_set_trajectory_device_rejects_bad_input(W):
    from paper_2102_00514_amd import binding as B
    pb = wl.config_c1()
    dm = _dev(pb.truth)
    with B.Smoother(pb, n_iter=2) as sm:
        with pytest.raises(B.SmootherError) as ei:
            sm.set_trajectory_device(dm.data_ptr(), 0, -np.eye(5))
        assert ei.value.status == B.SM_EINVAL
        with pytest.raises(B.SmootherError) as ei:
            sm.set_trajectory_device(0)
        assert ei.value.status == B.SM_EINVAL


def test_training_gains_over_prior_start(W):
    """Train the network on converged smoother outputs of 1024 seeded tracks
    (T = 4096) with the library's kernels, then start the smoother from it on
    64 held-out tracks: fewer iterations to a 1e-6 trajectory change than from
    the prior broadcast, to the same solution."""
    import torch
    net = _net(W, onn.DEFAULT, 1024, seed=0)
    X, LAB, stats = W.make_training_data(net, 1024, "taylor", chunk=1024, log=lambda *a: print(*a, flush=True))
    assert stats["kept"] >= 900
    mu, sigma = W.normalization(LAB)
    net.set_normalization(mu, sigma)
    hist, _ = W.train(net, X, LAB, epochs=3, batch=512, lr=2e-3, warmup=50, log_every=50,
                      log=lambda *a: print(*a, flush=True))
    assert hist[-1][1] < 0.5 * hist[0][1]
    cov, rmse = W.residual_covariance(net, X, LAB, sample=20000)
    assert np.all(np.linalg.eigvalsh(cov) > 0)
    del X, LAB
    pb = wl.config_c4(0, 64, held_out=True)
    r = W.time_to_converge(net, cov, pb, "taylor")
    print({k: v for k, v in W._public(r).items()}, flush=True)
    assert r["learned"]["iters_mean"] < r["plain"]["iters_mean"]
    assert r["learned"]["converged"] >= r["plain"]["converged"]
    assert r["distance_to_plain"]["tracks_within_1e-4"] >= 0.9
    net.close()
    torch.cuda.synchronize()


def test_mfma_trajectory_matches_oracle(W):
    """The inference form of the network (ws_trajectory_mfma: BF16 operands on
    the matrix cores, FP32 accumulation) with the trained weights on 16
    held-out tracks, against the oracle's forward with every weight and layer
    input rounded to bfloat16 (products and sums in FP64).

    The kernel rounds FP32 activations, the oracle FP64 ones, so an operand
    that lies within an FP32 ulp of a bfloat16 rounding boundary can round the
    other way: that moves a few outputs by up to about 2e-2 sigma (about 4 in
    1000 outputs by more than 1e-3 sigma), and the mean by about 1e-5 sigma.
    How often it happens depends on the order of the FP32 sums: an emulation
    of the residual kernel's order (tap-major, 16-product chunks) on the CPU
    gives mean 1.2e-5 and 3.5e-3 beyond 1e-3; the (channel, tap) order of the
    generic kernel 5.7e-6 and 1.6e-3.  Gates: mean below 5e-5 sigma, max below
    5e-2 sigma, at most 1% of outputs beyond 1e-3 sigma.  A wrong operand or result layout moves outputs by
    order one; BF16 rounding itself (the FP64 forward against the rounded one)
    moves them by 6e-3 sigma on average and 0.1 sigma at most, which the test
    prints.  The smoother started from either trajectory needs about the same
    iterations."""
    import os
    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(root, "paper_2102_00514_amd", "weights", "warmstart_ieks.npz")
    net, cov, _ = W.load(path, stream=torch.cuda.current_stream().cuda_stream)
    with np.load(path) as z:
        mu = np.asarray(z["mu"], dtype=np.float64)
        sigma = np.asarray(z["sigma"], dtype=np.float64)
    cfgd = onn.DEFAULT
    pb = wl.config_c4(0, 16, held_out=True)
    dy = _dev(pb.y)
    net.set_tracks(pb.offsets)
    t16 = torch.empty((pb.n_slots, pb.nx), dtype=torch.float64, device="cuda")
    net.trajectory(dy.data_ptr(), t16.data_ptr(), mfma=True)
    torch.cuda.synchronize()
    got = t16.cpu().numpy()
    x = onn.features(pb.y, pb.offsets, cfgd)
    theta = net.params().astype(np.float64)

    def traj(rnd):
        out, _ = onn.forward(theta, x, cfgd, operand_round=rnd)
        return onn.trajectory(onn.outputs_to_states(out, mu, sigma, cfgd), pb.offsets, cfgd)

    ref16, ref64 = traj(onn.bf16_round), traj(None)
    d = np.abs(got - ref16) / sigma
    q = np.abs(ref16 - ref64) / sigma
    print(f"mfma vs BF16-operand oracle: max {d.max():.3e}, mean {d.mean():.3e}, beyond 1e-3: {np.mean(d > 1e-3):.2e}; "
          f"BF16 rounding itself: max {q.max():.3e}, mean {q.mean():.3e} (units of sigma)", flush=True)
    assert np.all(np.isfinite(got))
    assert d.mean() < 5e-5 and d.max() < 5e-2 and np.mean(d > 1e-3) < 1e-2
    r32 = W.time_to_converge(net, cov, pb, "taylor")
    r16 = W.time_to_converge(net, cov, pb, "taylor", mfma=True)
    print(f"iterations: fp32 start {r32['learned']['iters_mean']:.2f}, mfma start {r16['learned']['iters_mean']:.2f}",
          flush=True)
    assert abs(r16["learned"]["iters_mean"] - r32["learned"]["iters_mean"]) <= 1.0
    net.close()
