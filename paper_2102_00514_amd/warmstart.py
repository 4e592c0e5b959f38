"""Learned initial trajectory for the iterated smoother.

ctypes binding of ``include/warmstart.h`` (the network's forward, backward and
Adam kernels live in ``libsmoother.so``), plus the pipeline around it:

* ``make_training_data`` simulates seeded tracks, runs the plain smoother
  (prior-broadcast start) on the GPU until every track's trajectory change is
  below ``tol`` or ``max_iter`` iterations have run, and turns the converged
  means into per-window labels; tracks that do not converge are dropped and
  counted;
* ``train`` runs Adam over shuffled mini-batches of windows;
* ``time_to_converge`` runs the smoother from the prior broadcast and from
  the network's trajectory and reports iterations and wall time to reach
  ``tol``, with the converged plain smoother as the reference.

PyTorch provides device memory and the stream only; the arithmetic runs in the
library's kernels.  ``python -m paper_2102_00514_amd.warmstart --help``.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time
from typing import Optional

import numpy as np

from . import binding
from . import workloads as wl

WS_OK, WS_EINVAL, WS_ENOMEM, WS_EDEVICE, _, WS_ESTATE = range(6)
WS_EXPORTS = ("ws_config_defaults", "ws_param_count", "ws_create", "ws_set_params", "ws_get_params",
              "ws_set_normalization", "ws_set_tracks", "ws_windows", "ws_labels", "ws_train_step",
              "ws_gradient", "ws_predict", "ws_trajectory", "ws_trajectory_mfma", "ws_last_error", "ws_destroy")

_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


class ws_config(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("patch", ctypes.c_int32), ("width", ctypes.c_int32),
                ("hidden", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("max_batch", ctypes.c_int32)]


class ws_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class WarmStartError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ws status {status}: {msg}")
        self.status = status


def _setup(lib):
    lib.ws_config_defaults.argtypes = [ctypes.POINTER(ws_config)]
    lib.ws_config_defaults.restype = None
    lib.ws_param_count.argtypes = [ctypes.POINTER(ws_config)]
    lib.ws_param_count.restype = ctypes.c_int64
    lib.ws_create.argtypes = [ctypes.POINTER(ws_config), _vp, ctypes.POINTER(_vp)]
    lib.ws_set_params.argtypes = [_vp, _fp, ctypes.c_int64]
    lib.ws_get_params.argtypes = [_vp, _fp, ctypes.c_int64]
    lib.ws_set_normalization.argtypes = [_vp, _fp, _fp]
    lib.ws_set_tracks.argtypes = [_vp, _i64p, ctypes.c_int32, _i64p]
    lib.ws_windows.argtypes = [_vp, _vp, _vp]
    lib.ws_labels.argtypes = [_vp, _vp, _vp]
    lib.ws_train_step.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, ctypes.c_int32, ctypes.POINTER(ws_adam), _fp]
    lib.ws_gradient.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, ctypes.c_int32, _fp, _fp]
    lib.ws_predict.argtypes = [_vp, _vp, ctypes.c_int64, _vp, ctypes.c_int32, _vp]
    lib.ws_trajectory.argtypes = [_vp, _vp, _vp]
    lib.ws_trajectory_mfma.argtypes = [_vp, _vp, _vp]
    for n in ("ws_create", "ws_set_params", "ws_get_params", "ws_set_normalization", "ws_set_tracks",
              "ws_windows", "ws_labels", "ws_train_step", "ws_gradient", "ws_predict", "ws_trajectory",
              "ws_trajectory_mfma"):
        getattr(lib, n).restype = ctypes.c_int
    lib.ws_last_error.argtypes = [_vp]
    lib.ws_last_error.restype = ctypes.c_char_p
    lib.ws_destroy.argtypes = [_vp]
    lib.ws_destroy.restype = None
    return lib


_lib = _setup(binding.lib())


def config(**overrides) -> ws_config:
    c = ws_config()
    _lib.ws_config_defaults(ctypes.byref(c))
    for k, v in overrides.items():
        setattr(c, k, int(v))
    return c


def config_dict(c: ws_config) -> dict:
    return {f: int(getattr(c, f)) for f, _ in ws_config._fields_}


def param_count(c: ws_config) -> int:
    return int(_lib.ws_param_count(ctypes.byref(c)))


def layer_shapes(c: ws_config):
    """[(weight shape, bias length)] in parameter order: embed, hidden layers, head."""
    out = [((c.width, 2 * c.ny, c.patch), c.width)]
    out += [((c.width, c.width, 3), c.width) for _ in range(c.hidden)]
    out += [((c.patch * c.nx, c.width), c.patch * c.nx)]
    return out


def init_params(c: ws_config, seed: int = 0) -> np.ndarray:
    """He-normal weights (standard deviation sqrt(2 / fan-in)), zero biases;
    the head is scaled by 0.1 so that the untrained network predicts about the
    label mean."""
    rng = np.random.default_rng(seed)
    parts = []
    shapes = layer_shapes(c)
    for li, (ws, nb) in enumerate(shapes):
        fan_in = int(np.prod(ws[1:]))
        std = np.sqrt(2.0 / fan_in) * (0.1 if li == len(shapes) - 1 else 1.0)
        parts.append(rng.standard_normal(int(np.prod(ws))) * std)
        parts.append(np.zeros(nb))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == param_count(c)
    return theta


class WarmStartNet:
    """One network handle (parameters, Adam state and workspace on the device)."""

    def __init__(self, cfg: Optional[ws_config] = None, stream: Optional[int] = None, params=None, seed: int = 0):
        self.cfg = cfg or config()
        h = _vp()
        st = _lib.ws_create(ctypes.byref(self.cfg), _vp(stream or 0), ctypes.byref(h))
        if st != WS_OK:
            raise WarmStartError(st, _lib.ws_last_error(None).decode())
        self.h = h.value
        self.n_params = param_count(self.cfg)
        self.n_windows = 0
        self.set_params(init_params(self.cfg, seed) if params is None else params)

    def _check(self, st):
        if st != WS_OK:
            raise WarmStartError(st, _lib.ws_last_error(self.h).decode())

    def set_params(self, theta) -> None:
        t = np.ascontiguousarray(theta, dtype=np.float32)
        self._check(_lib.ws_set_params(self.h, t.ctypes.data_as(_fp), t.size))

    def params(self) -> np.ndarray:
        t = np.empty(self.n_params, dtype=np.float32)
        self._check(_lib.ws_get_params(self.h, t.ctypes.data_as(_fp), t.size))
        return t

    def set_normalization(self, mu, sigma) -> None:
        m = np.ascontiguousarray(mu, dtype=np.float32)
        s = np.ascontiguousarray(sigma, dtype=np.float32)
        self.mu, self.sigma = m.copy(), s.copy()
        self._check(_lib.ws_set_normalization(self.h, m.ctypes.data_as(_fp), s.ctypes.data_as(_fp)))

    def set_tracks(self, offsets) -> int:
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n = ctypes.c_int64()
        self._check(_lib.ws_set_tracks(self.h, off.ctypes.data_as(_i64p), len(off) - 1, ctypes.byref(n)))
        self.n_windows = n.value
        return n.value

    def windows(self, y_ptr: int, x_ptr: int) -> None:
        self._check(_lib.ws_windows(self.h, _vp(y_ptr), _vp(x_ptr)))

    def labels(self, mean_ptr: int, lab_ptr: int) -> None:
        self._check(_lib.ws_labels(self.h, _vp(mean_ptr), _vp(lab_ptr)))

    def train_step(self, x_ptr: int, lab_ptr: int, n_data: int, idx_ptr: int, n: int, lr: float, beta1=0.9,
                   beta2=0.999, eps=1e-8, want_loss: bool = False):
        opt = ws_adam(lr, beta1, beta2, eps)
        loss = ctypes.c_float(0.0)
        self._check(_lib.ws_train_step(self.h, _vp(x_ptr), _vp(lab_ptr), n_data, _vp(idx_ptr), n,
                                       ctypes.byref(opt), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def gradient(self, x_ptr: int, lab_ptr: int, n_data: int, idx_ptr: int, n: int):
        g = np.empty(self.n_params, dtype=np.float32)
        loss = ctypes.c_float(0.0)
        self._check(_lib.ws_gradient(self.h, _vp(x_ptr), _vp(lab_ptr), n_data, _vp(idx_ptr), n,
                                     g.ctypes.data_as(_fp), ctypes.byref(loss)))
        return g, loss.value

    def predict(self, x_ptr: int, n_data: int, idx_ptr: int, n: int, states_ptr: int) -> None:
        self._check(_lib.ws_predict(self.h, _vp(x_ptr), n_data, _vp(idx_ptr), n, _vp(states_ptr)))

    def trajectory(self, y_ptr: int, mean_ptr: int, mfma: bool = False) -> None:
        """Initial trajectory of the planned tracks; mfma: BF16 products on the
        matrix cores (ws_trajectory_mfma) instead of the FP32 evaluation."""
        fn = _lib.ws_trajectory_mfma if mfma else _lib.ws_trajectory
        self._check(fn(self.h, _vp(y_ptr), _vp(mean_ptr)))

    def close(self):
        if getattr(self, "h", None):
            _lib.ws_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Pipeline (PyTorch for device memory only)
# ---------------------------------------------------------------------------

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the warm-start pipeline needs a GPU")
    return torch


def smooth_until_converged(pb: wl.Problem, stream: int, lin: str = "taylor", max_iter: int = 50,
                           tol: float = 1e-6, net: Optional["WarmStartNet"] = None, d_y=None, cov_const=None,
                           keep_mean: bool = True, schedule=(0, 0), freeze: bool = False,
                           mfma: bool = False) -> dict:
    """Runs the smoother on a batch until every track's trajectory change has
    been below tol once, or max_iter iterations (smoother_iterate_until).
    With ``net`` the first trajectory comes from the network (measurements d_y
    already on the device, tracks planned with ``net.set_tracks``).  Returns
    per-track iterations to converge (max_iter + 1 = not converged), the wall
    time from the first trajectory to the return of the driver, and the final
    means on the device.  ``schedule`` = (tile_lanes, lane_slots), 0 = automatic.
    With ``freeze`` a converged track is not iterated again (its result is its
    iterate at convergence) and tiles of converged tracks are skipped."""
    torch = _torch()
    sm = binding.Smoother(pb, stream=stream, n_iter=max_iter, lin=lin, tile_lanes=schedule[0],
                          lane_slots=schedule[1], freeze_converged=freeze)
    S, ntr, _ = sm.info()
    torch.cuda.synchronize()
    start = time.perf_counter()
    mean0 = None
    if net is not None:
        mean0 = torch.empty((S, pb.nx), dtype=torch.float64, device="cuda")
        net.trajectory(d_y.data_ptr(), mean0.data_ptr(), mfma=mfma)
        sm.set_trajectory_device(mean0.data_ptr(), 0, cov_const)
    run, first, finite = sm.iterate_until(tol, max_iter)
    wall = time.perf_counter() - start
    iters = np.where(first > 0, first, max_iter + 1).astype(np.int64)
    out = {"iters": iters, "wall_s": wall, "iterations_run": run, "finite": finite}
    if keep_mean:
        mean = torch.empty((S, pb.nx), dtype=torch.float64, device="cuda")
        sm.result_device(mean.data_ptr(), 0)
        torch.cuda.synchronize()
        out["mean"] = mean
    sm.close()
    return out


def _gen_chunk(args):
    first, count, held_out = args
    return wl.config_c4(first, count, held_out=held_out)


def generate(first: int, count: int, held_out: bool = False, chunk: int = 1024, workers: int = 1):
    """Seeded warm-start tracks first..first+count-1, in chunks (the tracks do
    not depend on the chunking)."""
    jobs = [(s, min(chunk, first + count - s), held_out) for s in range(first, first + count, chunk)]
    if workers <= 1:
        for j in jobs:
            yield _gen_chunk(j)
        return
    # The caller has usually initialised the GPU by now; HIP is not fork-safe,
    # so the workers are spawned (fresh interpreters that only simulate).
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        yield from ex.map(_gen_chunk, jobs)


def make_training_data(net: WarmStartNet, n_tracks: int, lin: str = "taylor", max_iter: int = 50,
                       tol: float = 1e-6, chunk: int = 4096, workers: int = 1, first: int = 0, log=print):
    """Inputs X [n_windows, 2 ny, W] and labels LAB [n_windows, W, nx] (device,
    float) of every converged track; returns (X, LAB, stats)."""
    torch = _torch()
    stream = torch.cuda.current_stream().cuda_stream
    xs, labs = [], []
    kept = dropped = 0
    iters_all = []
    t0 = time.perf_counter()
    for pb in generate(first, n_tracks, chunk=chunk, workers=workers):
        d_y = torch.from_numpy(np.ascontiguousarray(pb.y)).cuda()
        res = smooth_until_converged(pb, stream, lin, max_iter, tol)
        conv = res["iters"] <= max_iter
        iters_all.append(res["iters"])
        nw = net.set_tracks(pb.offsets)
        X = torch.empty((nw, 2 * pb.ny, net.cfg.window), dtype=torch.float32, device="cuda")
        LAB = torch.empty((nw, net.cfg.window, pb.nx), dtype=torch.float32, device="cuda")
        net.windows(d_y.data_ptr(), X.data_ptr())
        net.labels(res["mean"].data_ptr(), LAB.data_ptr())
        per_track = nw // pb.n_tracks if np.all(pb.lengths == pb.lengths[0]) else None
        if per_track is None:
            raise ValueError("training tracks must share one length")
        keep = torch.from_numpy(np.repeat(conv, per_track)).cuda()
        xs.append(X[keep])
        labs.append(LAB[keep])
        kept += int(conv.sum())
        dropped += int((~conv).sum())
        log(f"  tracks {kept + dropped}/{n_tracks}: kept {kept}, dropped {dropped} "
            f"(plain iterations median {np.median(res['iters']):.0f}), {time.perf_counter() - t0:.1f} s")
        del X, LAB, res, d_y
    its = np.concatenate(iters_all)
    stats = {"tracks": n_tracks, "kept": kept, "dropped_not_converged": dropped,
             "plain_iters_median": float(np.median(its)), "generation_s": time.perf_counter() - t0}
    return torch.cat(xs), torch.cat(labs), stats


def normalization(LAB, sample: int = 200_000, seed: int = 0):
    """Per-state mean and standard deviation of the labels (host, from a sample of windows)."""
    torch = _torch()
    n = LAB.shape[0]
    idx = np.random.default_rng(seed).choice(n, size=min(n, sample), replace=False)
    lab = LAB[torch.from_numpy(np.sort(idx)).cuda()].cpu().numpy().reshape(-1, LAB.shape[2]).astype(np.float64)
    return lab.mean(0).astype(np.float32), np.maximum(lab.std(0), 1e-6).astype(np.float32)


def train(net: WarmStartNet, X, LAB, epochs: int = 8, batch: int = 1024, lr: float = 1e-3, seed: int = 0,
          warmup: int = 200, lr_final: float = 0.02, log=print, log_every: int = 500):
    """Adam over shuffled mini-batches; learning rate: linear warm-up, then a
    cosine decay to lr * lr_final.  Returns the loss history (sampled)."""
    torch = _torch()
    n = X.shape[0]
    batch = min(batch, net.cfg.max_batch, n)
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    rng = np.random.default_rng(seed)
    hist = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).cuda()
        for b in range(steps_per_epoch):
            if step < warmup:
                lr_t = lr * (step + 1) / warmup
            else:
                u = (step - warmup) / max(1, total - warmup)
                lr_t = lr * (lr_final + (1 - lr_final) * 0.5 * (1 + np.cos(np.pi * u)))
            want = (step % log_every == 0) or step == total - 1
            idx_ptr = perm.data_ptr() + 4 * b * batch
            loss = net.train_step(X.data_ptr(), LAB.data_ptr(), n, idx_ptr, batch, lr_t, want_loss=want)
            if want:
                hist.append((step, loss))
                log(f"  epoch {ep} step {step}/{total} loss {loss:.5f} lr {lr_t:.2e} "
                    f"({time.perf_counter() - t0:.1f} s)")
            step += 1
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def residual_covariance(net: WarmStartNet, X, LAB, sample: int = 100_000, seed: int = 1):
    """Covariance of (prediction - label) over a sample of windows (host, FP64):
    the covariance given to the smoother with the network's first trajectory."""
    torch = _torch()
    n = X.shape[0]
    idx = np.sort(np.random.default_rng(seed).choice(n, size=min(n, sample), replace=False)).astype(np.int32)
    d_idx = torch.from_numpy(idx).cuda()
    pred = torch.empty((len(idx), net.cfg.window, net.cfg.nx), dtype=torch.float32, device="cuda")
    net.predict(X.data_ptr(), n, d_idx.data_ptr(), len(idx), pred.data_ptr())
    r = (pred - LAB[d_idx.long()]).cpu().numpy().reshape(-1, net.cfg.nx).astype(np.float64)
    return np.cov(r.T), float(np.sqrt(np.mean(r ** 2)))


def save(path: str, net: WarmStartNet, cov: np.ndarray, meta: dict) -> None:
    np.savez(path, params=net.params(), mu=net.mu, sigma=net.sigma, cov=cov,
             config=np.array(json.dumps(config_dict(net.cfg))), meta=np.array(json.dumps(meta)))


def load(path: str, stream: Optional[int] = None, max_batch: Optional[int] = None):
    """(net, residual covariance, meta) from a file written by ``save``."""
    with np.load(path, allow_pickle=False) as z:
        cfgd = json.loads(str(z["config"]))
        if max_batch:
            cfgd["max_batch"] = max_batch
        net = WarmStartNet(config(**cfgd), stream=stream, params=z["params"])
        net.set_normalization(z["mu"], z["sigma"])
        return net, np.array(z["cov"]), json.loads(str(z["meta"]))


def time_to_converge(net: WarmStartNet, cov: np.ndarray, pb: wl.Problem, lin: str = "taylor",
                     max_iter: int = 50, tol: float = 1e-6, repeats: int = 1, schedule=(0, 0),
                     mfma: bool = False) -> dict:
    """Plain (prior broadcast) vs learned first trajectory on the same tracks.

    A first run of each start gives the iterations per track to reach tol
    (max_iter + 1 = not converged) and the converged means; ``ms_to_converge``
    is then the best of ``repeats`` timed runs capped at the iteration where
    the last converging track converged (the learned runs include the
    network's inference -- FP32, or with ``mfma`` BF16 products on the matrix
    cores -- and the hand-over of its trajectory), and
    ``ms_to_converge_freeze`` the same with every converged track taken out
    of the later iterations (sm_problem.freeze_converged).  A start that
    brings one more slow track under tol pays for it in ``ms_to_converge``;
    ``ms_to_converge_common`` is capped instead at the iteration where the
    last of the tracks that both starts converge converged (the same set of
    tracks for both).  The distance of
    the learned run's converged means to the plain run's is reported per track
    (the plain smoother is the reference)."""
    torch = _torch()
    stream = torch.cuda.current_stream().cuda_stream
    d_y = torch.from_numpy(np.ascontiguousarray(pb.y)).cuda()
    net.set_tracks(pb.offsets)
    starts = (("plain", {}), ("learned", {"net": net, "d_y": d_y, "cov_const": cov, "mfma": mfma}))
    first = {}
    for name, kw in starts:
        first[name] = smooth_until_converged(pb, stream, lin, max_iter, tol, schedule=schedule, **kw)
    # tracks that both starts bring under tol: the like-for-like set
    common = (first["plain"]["iters"] <= max_iter) & (first["learned"]["iters"] <= max_iter)
    res = {}
    for name, kw in starts:
        kw = dict(kw, schedule=schedule)
        r = first[name]
        conv = r["iters"] <= max_iter
        kmax = int(r["iters"][conv].max()) if conv.any() else None
        kcom = int(r["iters"][common].max()) if common.any() else None

        def timed(k, freeze=False):
            if not k:
                return None
            return 1e3 * min(smooth_until_converged(pb, stream, lin, k, tol, keep_mean=False, freeze=freeze,
                                                    **kw)["wall_s"] for _ in range(repeats))

        ms = timed(kmax)
        res[name] = {"iters_mean": float(np.mean(r["iters"])), "iters_median": float(np.median(r["iters"])),
                     "iters_max_converged": kmax, "converged": float(conv.mean()),
                     "ms_to_converge": ms,
                     "ms_to_converge_freeze": timed(kmax, True) if pb.n_tracks > 1 else None,
                     "iters_max_common": kcom,
                     "ms_to_converge_common": ms if kcom == kmax else timed(kcom),
                     "ms_to_cap": 1e3 * r["wall_s"], "_mean": r["mean"], "_iters": r["iters"]}
    both = common
    so = pb.slot_offsets()
    diff = (res["learned"]["_mean"] - res["plain"]["_mean"]).abs().amax(dim=1).cpu().numpy()
    per_track = np.array([diff[so[i]:so[i + 1]].max() for i in range(pb.n_tracks)])
    res["distance_to_plain"] = {
        "max_over_tracks_converged_by_both": float(per_track[both].max()) if both.any() else None,
        "tracks_within_1e-4": float(np.mean(per_track[both] < 1e-4)) if both.any() else None}
    return res


def time_inference(net: WarmStartNet, pb: wl.Problem, repeats: int = 5) -> dict:
    """Wall time of the initial trajectory of every track of pb (features,
    network, scatter), FP32 and with BF16 products on the matrix cores: one
    warm-up call each, then the mean of `repeats` calls between two
    synchronisations."""
    torch = _torch()
    d_y = torch.from_numpy(np.ascontiguousarray(pb.y)).cuda()
    n_windows = net.set_tracks(pb.offsets)
    mean0 = torch.empty((pb.n_slots, pb.nx), dtype=torch.float64, device="cuda")
    out = {"tracks": pb.n_tracks, "windows": n_windows, "chunk_windows": net.cfg.max_batch}
    for name, mfma in (("fp32", False), ("bf16_mfma", True)):
        net.trajectory(d_y.data_ptr(), mean0.data_ptr(), mfma=mfma)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            net.trajectory(d_y.data_ptr(), mean0.data_ptr(), mfma=mfma)
        torch.cuda.synchronize()
        out[f"ms_{name}"] = round((time.perf_counter() - t0) * 1e3 / repeats, 3)
    return out


def _public(r: dict) -> dict:
    return {k: (_public(v) if isinstance(v, dict) else v) for k, v in r.items() if not k.startswith("_")}


def main(argv=None):
    ap = argparse.ArgumentParser(description="train / evaluate the learned initial trajectory")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--tracks", type=int, default=50_000)
    t.add_argument("--epochs", type=int, default=8)
    t.add_argument("--batch", type=int, default=1024)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--lin", default="taylor", choices=["taylor", "cubature"])
    t.add_argument("--workers", type=int, default=8)
    t.add_argument("--chunk", type=int, default=4096)
    t.add_argument("--out", required=True)
    t.add_argument("--eval-tracks", type=int, default=512)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--tracks", type=int, default=512)
    e.add_argument("--lin", default="taylor", choices=["taylor", "cubature"])
    i = sub.add_parser("infer", help="time the initial trajectory of held-out tracks (FP32 and BF16 MFMA)")
    i.add_argument("--weights", required=True)
    i.add_argument("--tracks", type=int, default=512)
    i.add_argument("--chunk", type=int, default=16384, help="windows per forward pass (max_batch)")
    i.add_argument("--repeats", type=int, default=5)
    a = ap.parse_args(argv)
    torch = _torch()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    if a.cmd == "train":
        net = WarmStartNet(config(max_batch=max(a.batch, 1024)), stream=stream, seed=0)
        log(f"network: {net.n_params} parameters, {config_dict(net.cfg)}")
        X, LAB, stats = make_training_data(net, a.tracks, a.lin, chunk=a.chunk, workers=a.workers, log=log)
        mu, sigma = normalization(LAB)
        net.set_normalization(mu, sigma)
        log(f"training windows: {X.shape[0]}; mu {mu}, sigma {sigma}")
        hist, train_s = train(net, X, LAB, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
        cov, rmse = residual_covariance(net, X, LAB)
        meta = dict(stats, lin=a.lin, epochs=a.epochs, batch=a.batch, lr=a.lr, train_s=train_s,
                    final_loss=hist[-1][1], train_rmse=rmse, windows=int(X.shape[0]))
        save(a.out, net, cov, meta)
        log(json.dumps(meta))
        del X, LAB
        pb = wl.config_c4(0, a.eval_tracks, held_out=True)
        print(json.dumps({"train": meta, "held_out": _public(time_to_converge(net, cov, pb, a.lin))}))
    elif a.cmd == "infer":
        net, _, _ = load(a.weights, stream=stream, max_batch=a.chunk)
        pb = wl.config_c4(0, a.tracks, held_out=True)
        print(json.dumps(time_inference(net, pb, a.repeats)))
        net.close()
    else:
        net, cov, meta = load(a.weights, stream=stream)
        pb = wl.config_c4(0, a.tracks, held_out=True)
        print(json.dumps(_public(time_to_converge(net, cov, pb, a.lin))))


if __name__ == "__main__":
    main()
