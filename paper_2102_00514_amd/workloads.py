"""Seeded synthetic inputs for the iterated smoother.

This module only produces problem instances: the coordinated-turn target with
bearings-only sensors used in the paper's experiment (Section 5), stacked
multi-target variants, ragged batches of independent tracks, and random
linear-Gaussian models for checks.  It holds no linearisation, filtering,
smoothing or scan arithmetic; it is the one module that both the GPU path
and the CPU oracle are fed from.

Problem layout (shared by every consumer):
  * ``y``        [sum_i T_i, ny]  measurements, track i occupies rows
                 ``offsets[i] .. offsets[i+1]-1`` (y_1 .. y_T of that track);
  * ``offsets``  [n_tracks+1] int64 measurement offsets;
  * ``m0``       [n_tracks, nx], ``P0`` [n_tracks, nx, nx] per-track prior;
  * ``Q``, ``R`` shared process / measurement noise covariances;
  * ``params``   model parameter block (see ``MODEL_*`` below);
  * ``truth``    [sum_i (T_i+1), nx] simulated states x_0 .. x_T per track.

Model parameter blocks:
  * ``MODEL_LINEAR``: ``[F (nx*nx), c (nx), H (ny*nx), d (ny)]`` row-major,
    i.e. x_k = F x_{k-1} + c + q,  y_k = H x_k + d + r.
  * ``MODEL_CT_BEARINGS``: ``[dt, (sx, sy, target) * ny]``; the state is
    ``nx/5`` stacked coordinated-turn blocks ``[px, py, vx, vy, omega]`` and
    sensor s measures the bearing ``atan2(py - sy, px - sx)`` of block
    ``target``.  Bearings are reported wrapped to [-pi, pi).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

MODEL_LINEAR = 0
MODEL_CT_BEARINGS = 1

# Constants of the paper's experiment as configured for this workload.
CT_DT = 0.01
CT_Q = 0.1          # continuous white-noise acceleration spectral density
CT_Q_OMEGA = 0.01   # turn-rate noise spectral density
CT_R_STD = 0.05     # bearing noise standard deviation
CT_SENSORS = ((-1.5, 0.5), (1.0, 1.0))
CT_M0 = (0.1, 0.2, 1.0, 0.0, 0.0)


@dataclass
class Problem:
    nx: int
    ny: int
    model: int
    params: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    m0: np.ndarray          # [n_tracks, nx]
    P0: np.ndarray          # [n_tracks, nx, nx]
    y: np.ndarray           # [sum T, ny]
    offsets: np.ndarray     # [n_tracks + 1] int64
    truth: Optional[np.ndarray] = None  # [sum (T+1), nx]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_tracks(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    @property
    def n_slots(self) -> int:
        return int(self.offsets[-1] + self.n_tracks)

    def slot_offsets(self) -> np.ndarray:
        """Start of each track in the state (slot) arrays: offsets[i] + i."""
        return self.offsets + np.arange(self.n_tracks + 1, dtype=np.int64)

    def track(self, i: int) -> "Problem":
        """Single-track view of track i (copies)."""
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        so = self.slot_offsets()
        truth = None if self.truth is None else self.truth[so[i]:so[i + 1]].copy()
        return Problem(self.nx, self.ny, self.model, self.params.copy(), self.Q.copy(),
                       self.R.copy(), self.m0[i:i + 1].copy(), self.P0[i:i + 1].copy(),
                       self.y[a:b].copy(), np.array([0, b - a], dtype=np.int64), truth,
                       f"{self.name}[{i}]", dict(self.meta))

    def prefix(self, T: int) -> "Problem":
        """Single-track problem truncated to its first T measurements."""
        assert self.n_tracks == 1 and 1 <= T <= int(self.offsets[1])
        truth = None if self.truth is None else self.truth[:T + 1].copy()
        return Problem(self.nx, self.ny, self.model, self.params.copy(), self.Q.copy(),
                       self.R.copy(), self.m0.copy(), self.P0.copy(), self.y[:T].copy(),
                       np.array([0, T], dtype=np.int64), truth, f"{self.name}[:{T}]",
                       dict(self.meta))


def wrap_angle(a):
    """Map angles to [-pi, pi)."""
    return a - 2.0 * np.pi * np.floor((a + np.pi) / (2.0 * np.pi))


def ct_process_noise(dt=CT_DT, q=CT_Q, q_omega=CT_Q_OMEGA, n_targets=1) -> np.ndarray:
    """Process noise of the coordinated-turn model: continuous white-noise
    acceleration on the velocities (spectral density q) and a random walk on
    the turn rate (spectral density q_omega), integrated over one step dt."""
    blk = np.zeros((5, 5))
    blk[0, 0] = blk[1, 1] = q * dt ** 3 / 3.0
    blk[0, 2] = blk[2, 0] = blk[1, 3] = blk[3, 1] = q * dt ** 2 / 2.0
    blk[2, 2] = blk[3, 3] = q * dt
    blk[4, 4] = q_omega * dt
    return np.kron(np.eye(n_targets), blk)


def _ct_propagate(X: np.ndarray, dt: float) -> np.ndarray:
    """Exact coordinated-turn motion over dt for rows of 5-vectors (simulator)."""
    px, py, vx, vy, w = (X[..., i] for i in range(5))
    a = w * dt
    small = np.abs(a) < 1e-4
    safe_w = np.where(small, 1.0, w)
    sin_a, cos_a = np.sin(a), np.cos(a)
    s1 = np.where(small, dt * (1.0 - a * a / 6.0), sin_a / safe_w)
    s2 = np.where(small, dt * (a / 2.0 - a ** 3 / 24.0), 2.0 * np.sin(a / 2.0) ** 2 / safe_w)
    out = np.empty_like(X)
    out[..., 0] = px + s1 * vx - s2 * vy
    out[..., 1] = py + s2 * vx + s1 * vy
    out[..., 2] = cos_a * vx - sin_a * vy
    out[..., 3] = sin_a * vx + cos_a * vy
    out[..., 4] = w
    return out


def ct_params(sensors, targets=None, dt=CT_DT) -> np.ndarray:
    sensors = np.asarray(sensors, dtype=np.float64).reshape(-1, 2)
    if targets is None:
        targets = np.zeros(len(sensors))
    blk = np.column_stack([sensors, np.asarray(targets, dtype=np.float64)])
    return np.concatenate([[dt], blk.ravel()])


def _simulate_ct(x0: np.ndarray, T: int, Lq: np.ndarray, proc: np.ndarray, meas: np.ndarray,
                 sensors: np.ndarray, targets: np.ndarray, dt: float, r_std: float):
    """One track: x_k = f(x_{k-1}) + Lq xi_k, y_k = wrap(h(x_k) + r_std zeta_k)."""
    nx = x0.shape[0]
    nt = nx // 5
    xs = np.empty((T + 1, nx))
    xs[0] = x0
    for k in range(1, T + 1):
        xs[k] = _ct_propagate(xs[k - 1].reshape(nt, 5), dt).ravel() + Lq @ proc[k - 1]
    tgt = targets.astype(np.int64)
    px = xs[1:, 5 * tgt]
    py = xs[1:, 5 * tgt + 1]
    ang = np.arctan2(py - sensors[:, 1], px - sensors[:, 0])
    y = wrap_angle(ang + r_std * meas)
    return xs, y


def ct_bearings(T: int, seed=0, m0=CT_M0, x0=None, sensors=CT_SENSORS) -> Problem:
    """Single coordinated-turn track observed by bearing sensors.

    The generator ``numpy.random.default_rng(seed)`` first draws the T x 5
    process noise and then the T x ny measurement noise; the true initial
    state defaults to the prior mean."""
    rng = np.random.default_rng(seed)
    sensors = np.asarray(sensors, dtype=np.float64)
    ny = sensors.shape[0]
    Q = ct_process_noise()
    R = CT_R_STD ** 2 * np.eye(ny)
    m0 = np.asarray(m0, dtype=np.float64)
    x0 = m0 if x0 is None else np.asarray(x0, dtype=np.float64)
    proc = rng.standard_normal((T, 5))
    meas = rng.standard_normal((T, ny))
    xs, y = _simulate_ct(x0, T, np.linalg.cholesky(Q), proc, meas, sensors,
                         np.zeros(ny), CT_DT, CT_R_STD)
    return Problem(5, ny, MODEL_CT_BEARINGS, ct_params(sensors), Q, R, m0[None].copy(),
                   np.eye(5)[None].copy(), y, np.array([0, T], dtype=np.int64), xs,
                   f"ct_bearings(T={T},seed={seed})")


def config_c1() -> Problem:
    """Coordinated turn + two bearings, T=100, seed 0."""
    return ct_bearings(100, seed=0)


def config_c2(T: int = 2 ** 15) -> Problem:
    """One 2^15-step seed-0 simulation; shorter lengths are its prefixes."""
    p = ct_bearings(2 ** 15, seed=0)
    return p if T == 2 ** 15 else p.prefix(T)


def _random_ct_state(rng) -> np.ndarray:
    px, py = rng.uniform(-1.0, 1.0, 2)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    w = rng.uniform(-1.0, 1.0)
    return np.array([px, py, np.cos(phi), np.sin(phi), w])


def ct_batch(n_tracks: int, t_min: int, t_max: int, seed_tag: int = 3,
             sensors=CT_SENSORS, first: int = 0, initial_state=None, prior_mean=None) -> Problem:
    """Ragged batch of independent coordinated-turn tracks.

    Track i uses ``default_rng([seed_tag, i])``: its length T_i ~ U{t_min..t_max}
    (no draw when t_min == t_max),
    its true initial state (uniform position, unit speed with uniform heading,
    turn rate ~ U(-1, 1)), then the process and measurement noise.  The prior
    mean is the true initial state with the turn rate set to zero, P0 = I.
    The tracks are propagated together, one time step for all live tracks at a
    time.

    ``first`` offsets the track index in the seed (tracks first..first+n-1);
    ``initial_state(rng)`` replaces the true-initial-state draw and
    ``prior_mean(x0)`` the prior rule."""
    sensors = np.asarray(sensors, dtype=np.float64)
    ny = sensors.shape[0]
    Q = ct_process_noise()
    Lq = np.linalg.cholesky(Q)
    R = CT_R_STD ** 2 * np.eye(ny)
    lengths = np.empty(n_tracks, dtype=np.int64)
    x0 = np.empty((n_tracks, 5))
    procs, meass = [], []
    for i in range(n_tracks):
        rng = np.random.default_rng([seed_tag, first + i])
        T = t_min if t_min == t_max else int(rng.integers(t_min, t_max + 1))
        x0[i] = (initial_state or _random_ct_state)(rng)
        procs.append(rng.standard_normal((T, 5)))
        meass.append(rng.standard_normal((T, ny)))
        lengths[i] = T
    tmax = int(lengths.max())
    states = np.empty((tmax + 1, n_tracks, 5))
    states[0] = x0
    noise = np.zeros((tmax, n_tracks, 5))
    for i in range(n_tracks):
        noise[:lengths[i], i] = procs[i] @ Lq.T
    for k in range(1, tmax + 1):
        states[k] = _ct_propagate(states[k - 1], CT_DT) + noise[k - 1]
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    ys, truths = [], []
    for i in range(n_tracks):
        T = int(lengths[i])
        xs = states[:T + 1, i]
        ang = np.arctan2(xs[1:, 1:2] - sensors[:, 1], xs[1:, 0:1] - sensors[:, 0])
        ys.append(wrap_angle(ang + CT_R_STD * meass[i]))
        truths.append(xs)
    if prior_mean is None:
        m0 = x0.copy()
        m0[:, 4] = 0.0
    else:
        m0 = np.stack([prior_mean(x) for x in x0])
    P0 = np.broadcast_to(np.eye(5), (n_tracks, 5, 5)).copy()
    return Problem(5, ny, MODEL_CT_BEARINGS, ct_params(sensors), Q, R, m0, P0,
                   np.concatenate(ys), offsets, np.concatenate(truths),
                   f"ct_batch({n_tracks},[{t_min},{t_max}])")


C4_T = 4096
C4_HELD_OUT_BASE = 10 ** 6


def _c4_initial_state(rng) -> np.ndarray:
    x0 = np.array(CT_M0, dtype=np.float64)
    x0[4] = rng.uniform(-1.0, 1.0)
    return x0


def config_c4(first: int, count: int, held_out: bool = False, T: int = C4_T) -> Problem:
    """Warm-start workload: tracks of T=4096 steps that all start from the
    experiment's initial position and velocity with a turn rate ~ U(-1, 1).
    Track i draws from ``default_rng([4, i])`` (training) or
    ``default_rng([4, 10^6 + i])`` (held out): the turn rate, then the process
    and measurement noise.  The prior is the single-track prior (turn rate 0,
    P0 = I) for every track."""
    base = C4_HELD_OUT_BASE if held_out else 0
    pb = ct_batch(count, T, T, seed_tag=4, first=base + first, initial_state=_c4_initial_state,
                  prior_mean=lambda x0: np.array(CT_M0, dtype=np.float64))
    pb.name = f"c4({'held-out' if held_out else 'train'} {first}..{first + count - 1}, T={T})"
    return pb


def config_c3(n_tracks: int = 4096, t_min: int = 100, t_max: int = 8192) -> Problem:
    return ct_batch(n_tracks, t_min, t_max, seed_tag=3)


def stacked_ct(T: int, rng, sensors=None, n_targets: int = 4, n_sensors: int = 8) -> Problem:
    """n_targets coordinated-turn targets stacked into one state; sensor s
    measures target s // (n_sensors // n_targets)."""
    if sensors is None:
        sensors = rng.uniform(-2.0, 2.0, (n_sensors, 2))
    per = n_sensors // n_targets
    targets = np.arange(n_sensors) // per
    nx = 5 * n_targets
    Q = ct_process_noise(n_targets=n_targets)
    R = CT_R_STD ** 2 * np.eye(n_sensors)
    x0 = np.concatenate([_random_ct_state(rng) for _ in range(n_targets)])
    proc = rng.standard_normal((T, nx))
    meas = rng.standard_normal((T, n_sensors))
    xs, y = _simulate_ct(x0, T, np.linalg.cholesky(Q), proc, meas, sensors, targets,
                         CT_DT, CT_R_STD)
    m0 = x0.copy()
    m0[4::5] = 0.0
    return Problem(nx, n_sensors, MODEL_CT_BEARINGS, ct_params(sensors, targets), Q, R,
                   m0[None], np.eye(nx)[None], y, np.array([0, T], dtype=np.int64), xs,
                   f"stacked_ct(T={T})", {"sensors": sensors})


def config_c5_single(T: int = 2 ** 16) -> Problem:
    """Four stacked coordinated-turn targets, eight bearing sensors drawn in
    [-2, 2]^2 from ``default_rng([5, 0])`` before the targets."""
    return stacked_ct(T, np.random.default_rng([5, 0]))


def config_c5_batch(n_tracks: int = 256, t_min: int = 1024, t_max: int = 2 ** 16) -> Problem:
    """Ragged batch of stacked tracks sharing the single-track sensor layout;
    track i draws its length and then, as ``stacked_ct``, its states and noises
    from ``default_rng([5, 1 + i])``.  The tracks are simulated together, one
    time step for all of them at once (the draws, and so the data, are those
    of ``stacked_ct`` track by track, up to the rounding of the noise
    products)."""
    n_targets, n_sensors = 4, 8
    sensors = np.random.default_rng([5, 0]).uniform(-2.0, 2.0, (n_sensors, 2))
    targets = np.arange(n_sensors) // (n_sensors // n_targets)
    nx = 5 * n_targets
    Q = ct_process_noise(n_targets=n_targets)
    Lq = np.linalg.cholesky(Q)
    Ts, x0s, procs, meass = [], [], [], []
    for i in range(n_tracks):
        rng = np.random.default_rng([5, 1 + i])
        T = int(rng.integers(t_min, t_max + 1))
        x0s.append(np.concatenate([_random_ct_state(rng) for _ in range(n_targets)]))
        procs.append(rng.standard_normal((T, nx)) @ Lq.T)
        meass.append(rng.standard_normal((T, n_sensors)))
        Ts.append(T)
    Tmax = max(Ts)
    noise = np.zeros((Tmax, n_tracks, nx))
    for i, p in enumerate(procs):
        noise[:Ts[i], i] = p
    X = np.empty((Tmax + 1, n_tracks, nx))
    X[0] = np.stack(x0s)
    for k in range(1, Tmax + 1):
        X[k] = _ct_propagate(X[k - 1].reshape(n_tracks, n_targets, 5), CT_DT).reshape(n_tracks, nx) + noise[k - 1]
    parts = []
    for i, T in enumerate(Ts):
        xs = X[:T + 1, i]
        px, py = xs[1:, 5 * targets], xs[1:, 5 * targets + 1]
        y = wrap_angle(np.arctan2(py - sensors[:, 1], px - sensors[:, 0]) + CT_R_STD * meass[i])
        m0 = xs[0].copy()
        m0[4::5] = 0.0
        parts.append(Problem(nx, n_sensors, MODEL_CT_BEARINGS, ct_params(sensors, targets), Q,
                             CT_R_STD ** 2 * np.eye(n_sensors), m0[None], np.eye(nx)[None], y,
                             np.array([0, T], dtype=np.int64), xs.copy(), f"stacked_ct(T={T})",
                             {"sensors": sensors}))
    return concat_tracks(parts, f"c5_batch({n_tracks})")


def concat_tracks(parts, name="batch") -> Problem:
    """Concatenate single-track problems that share the model, Q and R."""
    p0 = parts[0]
    lengths = np.array([int(p.offsets[-1]) for p in parts], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    truth = None
    if all(p.truth is not None for p in parts):
        truth = np.concatenate([p.truth for p in parts])
    return Problem(p0.nx, p0.ny, p0.model, p0.params.copy(), p0.Q.copy(), p0.R.copy(),
                   np.concatenate([p.m0 for p in parts]), np.concatenate([p.P0 for p in parts]),
                   np.concatenate([p.y for p in parts]), offsets, truth, name)


def random_spd(rng, n: int, scale: float = 1.0, cond: float = 10.0) -> np.ndarray:
    """Random symmetric positive-definite matrix with eigenvalues in [scale/cond, scale]."""
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = scale * np.exp(rng.uniform(np.log(1.0 / cond), 0.0, n))
    A = (U * ev) @ U.T
    return 0.5 * (A + A.T)


def linear_params(F, c, H, d) -> np.ndarray:
    return np.concatenate([np.ravel(F), np.ravel(c), np.ravel(H), np.ravel(d)]).astype(np.float64)


def linear_gaussian(nx: int, ny: int, T: int, seed: int = 0, n_tracks: int = 1,
                    t_min: Optional[int] = None) -> Problem:
    """Random stable linear-Gaussian model and simulated tracks.

    ``default_rng(seed)`` draws the model (F, c, H, d, Q, R, prior), then for each
    track its length (when ``t_min`` is given, T_i ~ U{t_min..T}), true initial state
    and noise."""
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((nx, nx))
    F *= 0.95 / max(1e-12, np.max(np.abs(np.linalg.eigvals(F))))
    c = 0.1 * rng.standard_normal(nx)
    H = rng.standard_normal((ny, nx))
    d = 0.1 * rng.standard_normal(ny)
    Q = random_spd(rng, nx, 0.1)
    R = random_spd(rng, ny, 0.2)
    m0 = rng.standard_normal(nx)
    P0 = random_spd(rng, nx, 1.0)
    Lq, Lr, L0 = (np.linalg.cholesky(M) for M in (Q, R, P0))
    ys, truths, lengths = [], [], []
    for _ in range(n_tracks):
        Ti = T if t_min is None else int(rng.integers(t_min, T + 1))
        x = m0 + L0 @ rng.standard_normal(nx)
        xs = [x]
        yk = []
        for _k in range(Ti):
            x = F @ x + c + Lq @ rng.standard_normal(nx)
            xs.append(x)
            yk.append(H @ x + d + Lr @ rng.standard_normal(ny))
        ys.append(np.array(yk).reshape(Ti, ny))
        truths.append(np.array(xs))
        lengths.append(Ti)
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    return Problem(nx, ny, MODEL_LINEAR, linear_params(F, c, H, d), Q, R,
                   np.tile(m0, (n_tracks, 1)), np.tile(P0, (n_tracks, 1, 1)),
                   np.concatenate(ys), offsets, np.concatenate(truths),
                   f"linear_gaussian({nx},{ny},T={T},seed={seed})",
                   {"F": F, "c": c, "H": H, "d": d})
