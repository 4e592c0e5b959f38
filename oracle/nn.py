"""Warm-start network oracle -- TEST INFRASTRUCTURE ONLY.

Plain NumPy FP64 definition of the learned initial-trajectory network (the
warm start that proposes the first linearisation trajectory, x̄^(0) of
Section 3, which the paper leaves to the user), its mean-squared-error loss,
the loss gradient by the chain rule, one Adam update (Kingma & Ba, 2015), and
the window / target / trajectory layouts that connect the network to the
smoother.  Only ``tests/`` may use it; the HIP library shares no code with it.

Network (one window of W measurement steps, channels first):
  input   x[c][t], c = 2*s + {0: sin, 1: cos} of bearing s, t = 0..W-1
  embed   z0[o][j] = b0[o] + sum_{c, u<P} W0[o][c][u] x[c][P j + u]      j = 0..W/P-1
          h0 = relu(z0)
  hidden  for l = 1..H (kernel 3, dilation d_l = 2^(l-1), zero outside the window):
          z_l[o][j] = b_l[o] + sum_{c, k<3} W_l[o][c][k] h_{l-1}[c][j + (k-1) d_l]
          h_l = h_{l-1} + relu(z_l)
  head    out[q][j] = bH[q] + sum_c WH[q][c] h_H[c][j],   q = u * nx + i
          -> normalised state i at step P j + u of the window
  state   = mu_i + sigma_i * out
  loss    = mean over (windows, steps, states) of (out - (label - mu) / sigma)^2

Parameters are one flat vector in the order W0, b0, (W_l, b_l) for l = 1..H,
WH, bH, each weight row-major over the index order written above.

Windows of a track with T measurements: n_w = ceil(T / W) windows; window w
starts at step 1 + W w, except the last, which starts at max(1, T - W + 1) so
that it ends at step T (steps past T, in a track shorter than W, repeat y_T).
Step k of the track is taken from window min((k-1) // W, n_w - 1); slot 0 (the
initial state) is given the network's estimate for step 1.

Reduced-precision inference: ``forward(..., operand_round=bf16_round)`` rounds
every weight and every layer input to bfloat16 before its products (the
products and sums stay in FP64, the bias, ReLU and residual in FP64 on the
unrounded values), which is what a product on BF16 matrix units with FP32
accumulation computes up to the order of its sums.
"""
from __future__ import annotations

import numpy as np

DEFAULT = dict(window=64, patch=4, width=128, hidden=4, nx=5, ny=2)


def layer_shapes(cfg=DEFAULT):
    """[(W shape, b shape)] for embed, hidden 1..H, head."""
    W, P, C, H, nx, ny = (cfg[k] for k in ("window", "patch", "width", "hidden", "nx", "ny"))
    assert W % P == 0
    shapes = [((C, 2 * ny, P), (C,))]
    shapes += [((C, C, 3), (C,)) for _ in range(H)]
    shapes += [((P * nx, C), (P * nx,))]
    return shapes


def n_params(cfg=DEFAULT) -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in layer_shapes(cfg))


def unpack(theta, cfg=DEFAULT):
    out, pos = [], 0
    for ws, bs in layer_shapes(cfg):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((theta[pos:pos + nw].reshape(ws), theta[pos + nw:pos + nw + nb].reshape(bs)))
        pos += nw + nb
    assert pos == theta.size
    return out


def init_params(rng, cfg=DEFAULT, dtype=np.float32):
    """He-normal weights (fan-in scaling), zero biases; the head is scaled down
    so that the untrained network predicts the label mean."""
    parts = []
    shapes = layer_shapes(cfg)
    for li, (ws, bs) in enumerate(shapes):
        fan_in = int(np.prod(ws[1:]))
        scale = np.sqrt(2.0 / fan_in) * (0.1 if li == len(shapes) - 1 else 1.0)
        parts.append(rng.standard_normal(int(np.prod(ws))) * scale)
        parts.append(np.zeros(int(np.prod(bs))))
    return np.concatenate(parts).astype(dtype)


def _dilated(h, k, d):
    """h[c][n][j + (k-1) d], zero where the index leaves the window."""
    L = h.shape[-1]
    off = (k - 1) * d
    out = np.zeros_like(h)
    if off >= 0:
        out[..., :L - off] = h[..., off:]
    else:
        out[..., -off:] = h[..., :L + off]
    return out


def bf16_round(a):
    """Nearest bfloat16 value (8 significant bits, ties to the even one) of
    each element of a, taken as an FP32 number first; returned as FP64.
    bfloat16 is the upper half of the IEEE binary32 encoding, so rounding adds
    half of the dropped 16-bit unit (minus one when the kept part is even, so
    that a tie goes to even) and clears the low 16 bits.  Finite inputs only."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, x, cfg=DEFAULT, operand_round=None):
    """x: [n, 2 ny, W] -> normalised outputs [n, P nx, W/P], cache for backward.
    operand_round: None, or a function applied to every weight and layer input
    before its products (bf16_round for the BF16 inference form)."""
    r = operand_round if operand_round is not None else (lambda v: v)
    P, H = cfg["patch"], cfg["hidden"]
    layers = unpack(np.asarray(theta, dtype=np.float64), cfg)
    n, cin, W = x.shape
    L = W // P
    patches = x.reshape(n, cin, L, P)                       # [n][c][j][u] = x[c][P j + u]
    W0, b0 = layers[0]
    z0 = np.einsum("ocu,ncju->noj", r(W0), r(patches)) + b0[None, :, None]
    h = np.maximum(z0, 0.0)
    cache = {"x": x, "h": [h], "a": [h]}
    for l in range(1, H + 1):
        Wl, bl = layers[l]
        d = 2 ** (l - 1)
        hr = r(h)
        z = bl[None, :, None] + sum(np.einsum("oc,ncj->noj", r(Wl[:, :, k]), _dilated(hr, k, d)) for k in range(3))
        a = np.maximum(z, 0.0)
        h = h + a
        cache["h"].append(h)
        cache["a"].append(a)
    WH, bH = layers[H + 1]
    out = np.einsum("qc,ncj->nqj", r(WH), r(h)) + bH[None, :, None]
    return out, cache


def outputs_to_states(out, mu, sigma, cfg=DEFAULT):
    """[n, P nx, W/P] normalised -> [n, W, nx] states."""
    n, _, L = out.shape
    P, nx = cfg["patch"], cfg["nx"]
    o = out.reshape(n, P, nx, L).transpose(0, 3, 1, 2).reshape(n, L * P, nx)
    return mu + sigma * o


def states_to_outputs(states, mu, sigma, cfg=DEFAULT):
    """Inverse of outputs_to_states: [n, W, nx] states -> normalised [n, P nx, W/P]."""
    n, W, nx = states.shape
    P = cfg["patch"]
    L = W // P
    o = ((states - mu) / sigma).reshape(n, L, P, nx).transpose(0, 2, 3, 1)
    return o.reshape(n, P * nx, L)


def loss(out, target):
    return float(np.mean((out - target) ** 2))


def backward(theta, cache, out, target, cfg=DEFAULT):
    """Gradient of ``loss`` with respect to the flat parameter vector."""
    P, H = cfg["patch"], cfg["hidden"]
    layers = unpack(np.asarray(theta, dtype=np.float64), cfg)
    grads = [None] * (H + 2)
    dout = 2.0 * (out - target) / out.size
    WH, _ = layers[H + 1]
    hH = cache["h"][H]
    grads[H + 1] = (np.einsum("nqj,ncj->qc", dout, hH), dout.sum(axis=(0, 2)))
    dh = np.einsum("qc,nqj->ncj", WH, dout)
    for l in range(H, 0, -1):
        Wl, _ = layers[l]
        d = 2 ** (l - 1)
        dz = dh * (cache["a"][l] > 0)
        hprev = cache["h"][l - 1]
        gW = np.stack([np.einsum("noj,ncj->oc", dz, _dilated(hprev, k, d)) for k in range(3)], axis=-1)
        grads[l] = (gW, dz.sum(axis=(0, 2)))
        # transpose of the dilated gather: h[j + (k-1)d] receives from z[j]
        dh = dh + sum(_dilated(np.einsum("oc,noj->ncj", Wl[:, :, k], dz), 2 - k, d) for k in range(3))
    dz0 = dh * (cache["a"][0] > 0)
    x = cache["x"]
    n, cin, W = x.shape
    patches = x.reshape(n, cin, W // P, P)
    grads[0] = (np.einsum("noj,ncju->ocu", dz0, patches), dz0.sum(axis=(0, 2)))
    return np.concatenate([np.concatenate([g.ravel(), b.ravel()]) for g, b in grads])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t = 1, 2, ...); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def window_table(offsets, W=DEFAULT["window"]):
    """[(track, first step)] of every window, tracks in order."""
    out = []
    for i in range(len(offsets) - 1):
        T = int(offsets[i + 1] - offsets[i])
        nw = -(-T // W)
        for w in range(nw):
            out.append((i, 1 + W * w if w < nw - 1 else max(1, T - W + 1)))
    return out


def features(y, offsets, cfg=DEFAULT):
    """Measurements [sum T, ny] -> network inputs [n_windows, 2 ny, W]."""
    W, ny = cfg["window"], cfg["ny"]
    tab = window_table(offsets, W)
    x = np.empty((len(tab), 2 * ny, W))
    for n, (i, st) in enumerate(tab):
        T = int(offsets[i + 1] - offsets[i])
        steps = np.minimum(st + np.arange(W), T)
        yy = y[offsets[i] + steps - 1]                        # [W][ny]
        x[n, 0::2] = np.sin(yy).T
        x[n, 1::2] = np.cos(yy).T
    return x


def window_labels(mean, offsets, cfg=DEFAULT):
    """Smoothed means [sum (T+1), nx] -> per-window labels [n_windows, W, nx]."""
    W = cfg["window"]
    tab = window_table(offsets, W)
    slot_off = np.concatenate([[0], np.cumsum(np.diff(offsets) + 1)])
    lab = np.empty((len(tab), W, cfg["nx"]))
    for n, (i, st) in enumerate(tab):
        T = int(offsets[i + 1] - offsets[i])
        steps = np.minimum(st + np.arange(W), T)
        lab[n] = mean[slot_off[i] + steps]
    return lab


def trajectory(states, offsets, cfg=DEFAULT):
    """Per-window states [n_windows, W, nx] -> initial trajectory [sum (T+1), nx]."""
    W = cfg["window"]
    tab = window_table(offsets, W)
    lengths = np.diff(offsets)
    slot_off = np.concatenate([[0], np.cumsum(lengths + 1)])
    out = np.full((int(slot_off[-1]), cfg["nx"]), np.nan)
    first = np.concatenate([[0], np.cumsum(-(-lengths // W))])
    for i in range(len(lengths)):
        T = int(lengths[i])
        nw = int(first[i + 1] - first[i])
        for k in range(1, T + 1):
            w = min((k - 1) // W, nw - 1)
            _, st = tab[first[i] + w]
            out[slot_off[i] + k] = states[first[i] + w, k - st]
        _, st0 = tab[first[i]]
        out[slot_off[i]] = states[first[i], 1 - st0]
    return out
