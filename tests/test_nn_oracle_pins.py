"""Pins of the warm-start network oracle against things other than itself:
torch's conv1d (a library routine for the same convolutions), torch autograd
and central finite differences (brute force) for the gradient, the closed form
of Adam's first steps, and invariants of the window layout."""
import numpy as np
import pytest

from oracle import nn

SMALL = dict(window=16, patch=4, width=6, hidden=2, nx=5, ny=2)


def _torch_forward(theta, x, cfg):
    import torch
    import torch.nn.functional as F
    layers = [(torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64)),
               torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)))
              for w, b in nn.unpack(np.asarray(theta, np.float64), cfg)]
    t = torch.from_numpy(x)
    W0, b0 = layers[0]
    h = torch.relu(F.conv1d(t, W0, b0, stride=cfg["patch"]))
    for l in range(1, cfg["hidden"] + 1):
        d = 2 ** (l - 1)
        Wl, bl = layers[l]
        h = h + torch.relu(F.conv1d(h, Wl, bl, padding=d, dilation=d))
    WH, bH = layers[-1]
    return F.conv1d(h, WH[:, :, None], bH), layers


@pytest.mark.parametrize("cfg", [SMALL, nn.DEFAULT])
def test_forward_matches_torch_conv1d(cfg):
    rng = np.random.default_rng(1)
    theta = nn.init_params(rng, cfg, dtype=np.float64)
    theta[-cfg["patch"] * cfg["nx"]:] = rng.standard_normal(cfg["patch"] * cfg["nx"])   # non-zero head bias
    x = rng.uniform(-1, 1, (3, 2 * cfg["ny"], cfg["window"]))
    out, _ = nn.forward(theta, x, cfg)
    ref, _ = _torch_forward(theta, x, cfg)
    assert out.shape == tuple(ref.shape)
    np.testing.assert_allclose(out, ref.numpy(), rtol=1e-12, atol=1e-12)


def test_param_count_default():
    # embed 128*4*4+128, 4 x (128*128*3+128), head 20*128+20
    assert nn.n_params() == 2176 + 4 * 49280 + 2580 == 201876


def _loss_at(theta, x, target, cfg):
    out, _ = nn.forward(theta, x, cfg)
    return nn.loss(out, target)


def test_gradient_finite_differences():
    rng = np.random.default_rng(2)
    cfg = SMALL
    theta = rng.standard_normal(nn.n_params(cfg)) * 0.4
    x = rng.uniform(-1, 1, (3, 4, cfg["window"]))
    target = rng.standard_normal((3, cfg["patch"] * cfg["nx"], cfg["window"] // cfg["patch"]))
    out, cache = nn.forward(theta, x, cfg)
    g = nn.backward(theta, cache, out, target, cfg)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (_loss_at(theta + e, x, target, cfg) - _loss_at(theta - e, x, target, cfg)) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-7 * np.max(np.abs(fd))


def test_gradient_matches_torch_autograd():
    import torch
    rng = np.random.default_rng(3)
    cfg = dict(SMALL, width=16, hidden=3, window=32)
    theta = rng.standard_normal(nn.n_params(cfg)) * 0.3
    x = rng.uniform(-1, 1, (5, 4, cfg["window"]))
    target = rng.standard_normal((5, cfg["patch"] * cfg["nx"], cfg["window"] // cfg["patch"]))
    out, cache = nn.forward(theta, x, cfg)
    g = nn.backward(theta, cache, out, target, cfg)
    ref, layers = _torch_forward(theta, x, cfg)
    for w, b in layers:
        w.requires_grad_(True)
        b.requires_grad_(True)
    import torch.nn.functional as F
    t = torch.from_numpy(x)
    hh = torch.relu(F.conv1d(t, *layers[0], stride=cfg["patch"]))
    for l in range(1, cfg["hidden"] + 1):
        d = 2 ** (l - 1)
        hh = hh + torch.relu(F.conv1d(hh, *layers[l], padding=d, dilation=d))
    o = F.conv1d(hh, layers[-1][0][:, :, None], layers[-1][1])
    torch.mean((o - torch.from_numpy(target)) ** 2).backward()
    gt = np.concatenate([np.concatenate([w.grad.numpy().ravel(), b.grad.numpy().ravel()]) for w, b in layers])
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-13)


def test_adam_first_steps_closed_form():
    # with bias correction the first step is lr * g / (|g| + eps); a second
    # step with the same gradient has m_hat = g and v_hat = g^2 again.
    rng = np.random.default_rng(4)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    th1, m, v = nn.adam_step(th, g, m, v, 1, lr, eps=eps)
    np.testing.assert_allclose(th1, th - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    th2, m, v = nn.adam_step(th1, g, m, v, 2, lr, eps=eps)
    np.testing.assert_allclose(th2, th1 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)


@pytest.mark.parametrize("lengths", [[1], [5, 64, 65], [128, 100, 63, 129]])
def test_window_table_covers_every_step(lengths):
    W = nn.DEFAULT["window"]
    offsets = np.concatenate([[0], np.cumsum(lengths)])
    tab = nn.window_table(offsets, W)
    for i, T in enumerate(lengths):
        starts = [st for tr, st in tab if tr == i]
        assert len(starts) == -(-T // W)
        assert starts[-1] + W - 1 == max(T, W)       # the last window ends at step T (or is padded)
        covered = set()
        for st in starts:
            covered.update(range(st, min(st + W, T + 1)))
        assert covered == set(range(1, T + 1))


def test_features_encode_the_bearings():
    rng = np.random.default_rng(5)
    lengths = [70, 64, 3]
    offsets = np.concatenate([[0], np.cumsum(lengths)])
    y = rng.uniform(-np.pi, np.pi, (offsets[-1], 2))
    x = nn.features(y, offsets)
    tab = nn.window_table(offsets)
    for n, (i, st) in enumerate(tab):
        T = lengths[i]
        for t in (0, 17, 63):
            k = min(st + t, T)
            for s in range(2):
                ang = np.arctan2(x[n, 2 * s, t], x[n, 2 * s + 1, t])
                assert abs(ang - y[offsets[i] + k - 1, s]) < 1e-12


def test_labels_and_trajectory_round_trip():
    rng = np.random.default_rng(6)
    lengths = np.array([200, 64, 7, 129])
    offsets = np.concatenate([[0], np.cumsum(lengths)])
    S = int((lengths + 1).sum())
    mean = rng.standard_normal((S, 5))
    lab = nn.window_labels(mean, offsets)
    traj = nn.trajectory(lab, offsets)
    so = np.concatenate([[0], np.cumsum(lengths + 1)])
    for i in range(len(lengths)):
        np.testing.assert_array_equal(traj[so[i] + 1:so[i + 1]], mean[so[i] + 1:so[i + 1]])
        np.testing.assert_array_equal(traj[so[i]], mean[so[i] + 1])


def test_output_state_maps_are_inverse():
    rng = np.random.default_rng(7)
    st = rng.standard_normal((4, 64, 5))
    mu, sigma = rng.standard_normal(5), rng.uniform(0.5, 2, 5)
    o = nn.states_to_outputs(st, mu, sigma)
    np.testing.assert_allclose(nn.outputs_to_states(o, mu, sigma), st, rtol=1e-14, atol=1e-14)
    # head channel q = u * nx + i at patch j is step P j + u, state i
    assert o[1, 2 * 5 + 3, 5] == pytest.approx((st[1, 4 * 5 + 2, 3] - mu[3]) / sigma[3])


def test_bf16_round_matches_torch():
    """bf16_round against torch's float32 -> bfloat16 conversion (round to
    nearest, ties to even), over many magnitudes and on exact ties."""
    import torch
    rng = np.random.default_rng(11)
    v = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000)).astype(np.float32)
    # exact ties: the dropped half is 0x8000, with the kept part even and odd
    kept = rng.integers(0x3F00, 0x4300, 400, dtype=np.uint32) << 16
    ties = (kept | 0x8000).view(np.float32)
    v = np.concatenate([v, ties, -ties, np.float32([0.0, -0.0, 1.0, 65504.0, 3.0e38])])
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = nn.bf16_round(v)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    # a tie goes to the even neighbour, so half of them round up
    up = nn.bf16_round(ties) > ties
    assert 0.3 < up.mean() < 0.7


def test_bf16_forward_matches_torch_conv1d():
    """The BF16-operand forward against torch's conv1d with every weight and
    every layer input rounded by torch's own bfloat16 conversion."""
    import torch
    import torch.nn.functional as F
    cfg = SMALL
    rng = np.random.default_rng(12)
    theta = nn.init_params(rng, cfg, dtype=np.float64)
    theta[-cfg["patch"] * cfg["nx"]:] = rng.standard_normal(cfg["patch"] * cfg["nx"])
    x = rng.uniform(-1, 1, (5, 2 * cfg["ny"], cfg["window"]))

    def rb(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    layers = [(torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64)),
               torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)))
              for w, b in nn.unpack(theta, cfg)]
    W0, b0 = layers[0]
    h = torch.relu(F.conv1d(rb(torch.from_numpy(x)), rb(W0), b0, stride=cfg["patch"]))
    for l in range(1, cfg["hidden"] + 1):
        d = 2 ** (l - 1)
        Wl, bl = layers[l]
        h = h + torch.relu(F.conv1d(rb(h), rb(Wl), bl, padding=d, dilation=d))
    WH, bH = layers[-1]
    want = F.conv1d(rb(h), rb(WH)[:, :, None], bH).numpy()
    got, _ = nn.forward(theta, x, cfg, operand_round=nn.bf16_round)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
    # and it is not the FP64 forward
    exact, _ = nn.forward(theta, x, cfg)
    assert np.max(np.abs(got - exact)) > 1e-4 * np.max(np.abs(exact))
