"""Thin ctypes binding of ``libsmoother.so`` (include/smoother.h).

Argument marshalling only: every step of the smoother runs in the HIP
library.  If the library is missing, importing this module raises -- there is
no fallback path.  PyTorch supplies device memory (result buffers) and the
HIP stream the work is queued on.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .workloads import Problem

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsmoother.so")

SM_OK, SM_EINVAL, SM_ENOMEM, SM_EDEVICE, SM_ENUMERIC, SM_ESTATE = range(6)
STATUS_NAMES = {0: "SM_OK", 1: "SM_EINVAL", 2: "SM_ENOMEM", 3: "SM_EDEVICE", 4: "SM_ENUMERIC", 5: "SM_ESTATE"}
SM_MODEL_LINEAR, SM_MODEL_CT_BEARINGS = 0, 1
LIN = {"taylor": 0, "cubature": 1, "unscented": 2}
PRECISION = {"f64": 0, "f32": 1}
SCAN = {"parallel": 0, "sequential": 1}
FORM = {"covariance": 0, "sqrt": 1}

EXPORTS = ("smoother_problem_defaults", "smoother_init", "smoother_iterate", "smoother_result",
           "smoother_result_device", "smoother_track_deltas", "smoother_info", "smoother_last_error",
           "smoother_destroy", "smoother_version", "smoother_profile", "smoother_schedule",
           "smoother_set_trajectory_device", "smoother_iterate_until", "smoother_autotune",
           "smoother_objective", "smoother_iterate_lm", "smoother_filter", "smoother_solve_static",
           "smoother_profile_repeat", "smoother_autotune_cached", "smoother_autotune_cache_clear")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


class sm_problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("n_tracks", ctypes.c_int32),
        ("offsets", _i64p),
        ("model", ctypes.c_int32), ("params", _dp), ("n_params", ctypes.c_int32),
        ("Q", _dp), ("R", _dp), ("m0", _dp), ("P0", _dp), ("y", _dp),
        ("n_iter", ctypes.c_int32), ("lin", ctypes.c_int32),
        ("ut_alpha", ctypes.c_double), ("ut_beta", ctypes.c_double), ("ut_kappa", ctypes.c_double),
        ("precision", ctypes.c_int32), ("scan", ctypes.c_int32),
        ("init_mean", _dp), ("init_cov", _dp),
        ("max_device_bytes", ctypes.c_int64),
        ("tile_lanes", ctypes.c_int32), ("lane_slots", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("lm_lambda", ctypes.c_double),
        ("form", ctypes.c_int32),
        ("freeze_converged", ctypes.c_int32),
    ]


class sm_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("positions", ctypes.c_int64)]


class SmootherError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (python -m paper_2102_00514_amd.build)")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (soname
    # libamdhip64.so.7) and requests it by the unversioned name, so if this
    # library were loaded first, PyTorch would map a second copy of the HIP and
    # HSA runtimes next to ours and ours would find no device.  Loading PyTorch
    # first lets this library's libamdhip64.so.7 dependency resolve to the
    # runtime PyTorch already holds.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.smoother_problem_defaults.argtypes = [ctypes.POINTER(sm_problem)]
    lib.smoother_problem_defaults.restype = None
    lib.smoother_init.argtypes = [ctypes.POINTER(sm_problem), vp, ctypes.POINTER(vp)]
    lib.smoother_init.restype = ctypes.c_int
    lib.smoother_iterate.argtypes = [vp, ctypes.c_int32, _dp, ctypes.POINTER(ctypes.c_int32)]
    lib.smoother_iterate.restype = ctypes.c_int
    lib.smoother_result.argtypes = [vp, _dp, _dp]
    lib.smoother_result.restype = ctypes.c_int
    lib.smoother_result_device.argtypes = [vp, vp, vp]
    lib.smoother_result_device.restype = ctypes.c_int
    lib.smoother_track_deltas.argtypes = [vp, _dp]
    lib.smoother_track_deltas.restype = ctypes.c_int
    lib.smoother_info.argtypes = [vp, _i64p, ctypes.POINTER(ctypes.c_int32), _i64p]
    lib.smoother_info.restype = ctypes.c_int
    lib.smoother_last_error.argtypes = [vp]
    lib.smoother_last_error.restype = ctypes.c_char_p
    lib.smoother_destroy.argtypes = [vp]
    lib.smoother_destroy.restype = None
    lib.smoother_profile.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(sm_kernel_time), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)]
    lib.smoother_profile.restype = ctypes.c_int
    lib.smoother_profile_repeat.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(sm_kernel_time),
                                            ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.smoother_profile_repeat.restype = ctypes.c_int
    lib.smoother_schedule.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _i64p]
    lib.smoother_schedule.restype = ctypes.c_int
    lib.smoother_version.argtypes = []
    lib.smoother_version.restype = ctypes.c_char_p
    lib.smoother_set_trajectory_device.argtypes = [vp, vp, vp, _dp]
    lib.smoother_set_trajectory_device.restype = ctypes.c_int
    lib.smoother_iterate_until.argtypes = [vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]
    lib.smoother_iterate_until.restype = ctypes.c_int
    lib.smoother_autotune.argtypes = [ctypes.POINTER(sm_problem), vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), _dp]
    lib.smoother_autotune.restype = ctypes.c_int
    lib.smoother_autotune_cached.argtypes = [ctypes.POINTER(sm_problem), vp, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _dp,
                                             ctypes.POINTER(ctypes.c_int32)]
    lib.smoother_autotune_cached.restype = ctypes.c_int
    lib.smoother_autotune_cache_clear.argtypes = []
    lib.smoother_autotune_cache_clear.restype = None
    lib.smoother_filter.argtypes = [vp, _dp, _dp, _dp]
    lib.smoother_filter.restype = ctypes.c_int
    lib.smoother_objective.argtypes = [vp, _dp]
    lib.smoother_objective.restype = ctypes.c_int
    lib.smoother_iterate_lm.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _dp]
    lib.smoother_iterate_lm.restype = ctypes.c_int
    lib.smoother_solve_static.argtypes = [ctypes.POINTER(sm_problem), vp, vp, vp, _dp]
    lib.smoother_solve_static.restype = ctypes.c_int
    return lib


_lib = _load()


def lib():
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(h, st):
    if st != SM_OK:
        raise SmootherError(st, smoother_last_error(h))


def smoother_last_error(h=None) -> str:
    return _lib.smoother_last_error(h).decode()


def make_problem(pb: Problem, n_iter: int = 10, lin: str = "taylor", precision: str = "f64",
                 scan: str = "parallel", init_mean=None, init_cov=None, ut_alpha=1.0, ut_beta=0.0,
                 ut_kappa=1.0, max_device_bytes: int = 0, tile_lanes: int = 0, lane_slots: int = 0,
                 use_graph: bool = True, lm_lambda: float = 0.0, form: str = "covariance",
                 freeze_converged: bool = False):
    """sm_problem for a workloads.Problem; returns (struct, keep-alive arrays)."""
    s = sm_problem()
    _lib.smoother_problem_defaults(ctypes.byref(s))
    keep = {
        "offsets": np.ascontiguousarray(pb.offsets, dtype=np.int64),
        "params": _f64(pb.params), "Q": _f64(pb.Q), "R": _f64(pb.R),
        "m0": _f64(pb.m0), "P0": _f64(pb.P0), "y": _f64(pb.y),
    }
    if init_mean is not None:
        keep["init_mean"] = _f64(init_mean)
    if init_cov is not None:
        keep["init_cov"] = _f64(init_cov)
    s.nx, s.ny, s.n_tracks = pb.nx, pb.ny, pb.n_tracks
    s.offsets = keep["offsets"].ctypes.data_as(_i64p)
    s.model = pb.model
    s.params, s.n_params = keep["params"].ctypes.data_as(_dp), keep["params"].size
    for k in ("Q", "R", "m0", "P0", "y"):
        setattr(s, k, keep[k].ctypes.data_as(_dp))
    s.n_iter = n_iter
    s.lin = LIN[lin]
    s.ut_alpha, s.ut_beta, s.ut_kappa = ut_alpha, ut_beta, ut_kappa
    s.precision = PRECISION[precision]
    s.scan = SCAN[scan]
    if "init_mean" in keep:
        s.init_mean = keep["init_mean"].ctypes.data_as(_dp)
    if "init_cov" in keep:
        s.init_cov = keep["init_cov"].ctypes.data_as(_dp)
    s.max_device_bytes = max_device_bytes
    s.tile_lanes, s.lane_slots = tile_lanes, lane_slots
    s.use_graph = int(bool(use_graph))
    s.lm_lambda = lm_lambda
    s.form = FORM[form]
    s.freeze_converged = int(bool(freeze_converged))
    return s, keep


def smoother_init(pb: Problem, stream: Optional[int] = None, **kw) -> int:
    """Creates a handle; ``stream`` is a HIP stream handle (torch's
    ``torch.cuda.current_stream().cuda_stream``), None = default stream."""
    s, _keep = make_problem(pb, **kw)
    h = ctypes.c_void_p()
    st = _lib.smoother_init(ctypes.byref(s), ctypes.c_void_p(stream or 0), ctypes.byref(h))
    if st != SM_OK:
        raise SmootherError(st, smoother_last_error(None))
    return h.value


def smoother_autotune(pb: Problem, stream: Optional[int] = None, iters: int = 5, **kw):
    """Fastest scan schedule for this problem: (tile_lanes, lane_slots, ms per iteration)."""
    s, _keep = make_problem(pb, **kw)
    B, K, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    st = _lib.smoother_autotune(ctypes.byref(s), ctypes.c_void_p(stream or 0), iters, ctypes.byref(B),
                                ctypes.byref(K), ctypes.byref(ms))
    if st != SM_OK:
        raise SmootherError(st, smoother_last_error(None))
    return B.value, K.value, ms.value


def smoother_autotune_cached(pb: Problem, stream: Optional[int] = None, iters: int = 5, **kw):
    """As smoother_autotune through the library's per-process cache of schedules
    by problem shape: (tile_lanes, lane_slots, ms per iteration, from_cache)."""
    s, _keep = make_problem(pb, **kw)
    B, K, ms, hit = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
    st = _lib.smoother_autotune_cached(ctypes.byref(s), ctypes.c_void_p(stream or 0), iters, ctypes.byref(B),
                                       ctypes.byref(K), ctypes.byref(ms), ctypes.byref(hit))
    if st != SM_OK:
        raise SmootherError(st, smoother_last_error(None))
    return B.value, K.value, ms.value, bool(hit.value)


def smoother_autotune_cache_clear() -> None:
    _lib.smoother_autotune_cache_clear()


def smoother_solve_static(pb: Problem, mean_ptr: int, cov_ptr: int, stream: Optional[int] = None,
                          want_delta: bool = True, **kw):
    """All n_iter iterations from the prior broadcast into caller-owned device
    buffers, with no device allocation (the library's static scratch); returns
    the last iteration's largest change (None without want_delta)."""
    s, _keep = make_problem(pb, **kw)
    d = ctypes.c_double()
    st = _lib.smoother_solve_static(ctypes.byref(s), ctypes.c_void_p(stream or 0), ctypes.c_void_p(mean_ptr),
                                    ctypes.c_void_p(cov_ptr), ctypes.byref(d) if want_delta else None)
    if st != SM_OK:
        raise SmootherError(st, smoother_last_error(None))
    return d.value if want_delta else None


def smoother_iterate(h: int, k: int = 0, want_delta: bool = True):
    """Runs k iterations (k <= 0: up to n_iter).  Returns (max_delta or None, iterations done)."""
    d = ctypes.c_double(0.0)
    it = ctypes.c_int32(0)
    st = _lib.smoother_iterate(h, k, ctypes.byref(d) if want_delta else None, ctypes.byref(it))
    if st == SM_ENUMERIC:
        return float("nan"), it.value
    _check(h, st)
    return (d.value if want_delta else None), it.value


def smoother_iterate_until(h: int, tol: float, max_iter: int):
    """Iterates until every track's trajectory change has been below tol once
    (or max_iter iterations).  Returns (iterations run, per-track first
    converged iteration, 0 = not converged, numerics ok)."""
    _, T, _ = smoother_info(h)
    run = ctypes.c_int32(0)
    first = np.zeros(T, dtype=np.int32)
    st = _lib.smoother_iterate_until(h, tol, max_iter, ctypes.byref(run),
                                     first.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if st == SM_ENUMERIC:
        return run.value, first, False
    _check(h, st)
    return run.value, first, True


def smoother_filter(h: int, nx: int, moments: bool = True):
    """One filtering pass at the current trajectory: (filtered means [S, nx],
    covariances [S, nx, nx]) or (None, None), and log p(y_{1:T}) per track."""
    S, T, _ = smoother_info(h)
    ll = np.empty(T)
    mean = np.empty((S, nx)) if moments else None
    cov = np.empty((S, nx, nx)) if moments else None
    _check(h, _lib.smoother_filter(h, None if mean is None else mean.ctypes.data_as(_dp),
                                   None if cov is None else cov.ctypes.data_as(_dp), ll.ctypes.data_as(_dp)))
    return mean, cov, ll


def smoother_objective(h: int) -> np.ndarray:
    """MAP objective of the current trajectory, per track."""
    _, T, _ = smoother_info(h)
    out = np.empty(T)
    _check(h, _lib.smoother_objective(h, out.ctypes.data_as(_dp)))
    return out


def smoother_iterate_lm(h: int, lambda0: float = 1e-2, nu: float = 10.0, tol: float = 1e-6, max_iter: int = 50):
    """Levenberg-Marquardt passes with Marquardt's damping schedule until every
    track has converged (or max_iter).  Returns (passes run, per-track pass of
    convergence (0 = none), per-track final objective); a failed track (not
    finite from the start) shows as a non-finite objective."""
    _, T, _ = smoother_info(h)
    run = ctypes.c_int32(0)
    first = np.zeros(T, dtype=np.int32)
    cost = np.empty(T)
    st = _lib.smoother_iterate_lm(h, lambda0, nu, tol, max_iter, ctypes.byref(run),
                                  first.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cost.ctypes.data_as(_dp))
    if st != SM_ENUMERIC:
        _check(h, st)
    return run.value, first, cost


def smoother_info(h: int):
    S, T, B = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(h, _lib.smoother_info(h, ctypes.byref(S), ctypes.byref(T), ctypes.byref(B)))
    return S.value, T.value, B.value


def smoother_result(h: int, nx: int):
    """Host copy of the current trajectory: mean [S, nx], cov [S, nx, nx]."""
    S, _, _ = smoother_info(h)
    mean = np.empty((S, nx))
    cov = np.empty((S, nx, nx))
    _check(h, _lib.smoother_result(h, mean.ctypes.data_as(_dp), cov.ctypes.data_as(_dp)))
    return mean, cov


def smoother_result_device(h: int, mean_ptr: int, cov_ptr: int) -> None:
    """Writes the trajectory into caller-owned device buffers (e.g. torch tensors' data_ptr())."""
    _check(h, _lib.smoother_result_device(h, ctypes.c_void_p(mean_ptr), ctypes.c_void_p(cov_ptr)))


def smoother_set_trajectory_device(h: int, mean_ptr: int, cov_ptr: int = 0, cov_const=None) -> None:
    """Next linearisation trajectory from device memory: means at mean_ptr,
    covariances at cov_ptr, else the constant host matrix cov_const, else P0."""
    cc = None if cov_const is None else _f64(cov_const)
    _check(h, _lib.smoother_set_trajectory_device(h, ctypes.c_void_p(mean_ptr), ctypes.c_void_p(cov_ptr or 0),
                                                  None if cc is None else cc.ctypes.data_as(_dp)))


def smoother_track_deltas(h: int) -> np.ndarray:
    _, T, _ = smoother_info(h)
    out = np.empty(T)
    _check(h, _lib.smoother_track_deltas(h, out.ctypes.data_as(_dp)))
    return out


def smoother_profile(h: int, k: int, repeat: int = 1) -> dict:
    """Runs k iterations with per-launch HIP events (each launch repeated
    `repeat` times between its events, the mean taken); returns
    {kernel family: (launches, total_ms, positions)}."""
    cap = 64
    recs = (sm_kernel_time * cap)()
    n = ctypes.c_int32(0)
    if repeat == 1:
        _check(h, _lib.smoother_profile(h, k, recs, cap, ctypes.byref(n)))
    else:
        _check(h, _lib.smoother_profile_repeat(h, k, repeat, recs, cap, ctypes.byref(n)))
    return {recs[i].name.decode(): (recs[i].launches, recs[i].total_ms, recs[i].positions) for i in range(n.value)}


def smoother_schedule(h: int):
    """(lanes per tile, slots per lane, tiles) of the scan schedule in use."""
    B, K, T = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(h, _lib.smoother_schedule(h, ctypes.byref(B), ctypes.byref(K), ctypes.byref(T)))
    return B.value, K.value, T.value


def smoother_destroy(h: int) -> None:
    _lib.smoother_destroy(h)


def smoother_version() -> str:
    return _lib.smoother_version().decode()


class Smoother:
    """Owning wrapper around one handle (same calls, context-managed)."""

    def __init__(self, pb: Problem, stream: Optional[int] = None, **kw):
        self.nx = pb.nx
        self.h = smoother_init(pb, stream, **kw)

    def iterate(self, k: int = 0, want_delta: bool = True):
        return smoother_iterate(self.h, k, want_delta)

    def result(self):
        return smoother_result(self.h, self.nx)

    def result_device(self, mean_ptr: int, cov_ptr: int):
        smoother_result_device(self.h, mean_ptr, cov_ptr)

    def track_deltas(self):
        return smoother_track_deltas(self.h)

    def iterate_until(self, tol: float, max_iter: int):
        return smoother_iterate_until(self.h, tol, max_iter)

    def objective(self):
        return smoother_objective(self.h)

    def filter(self, moments: bool = True):
        return smoother_filter(self.h, self.nx, moments)

    def iterate_lm(self, lambda0: float = 1e-2, nu: float = 10.0, tol: float = 1e-6, max_iter: int = 50):
        return smoother_iterate_lm(self.h, lambda0, nu, tol, max_iter)

    def set_trajectory_device(self, mean_ptr: int, cov_ptr: int = 0, cov_const=None):
        smoother_set_trajectory_device(self.h, mean_ptr, cov_ptr, cov_const)

    def info(self):
        return smoother_info(self.h)

    def profile(self, k: int, repeat: int = 1):
        return smoother_profile(self.h, k, repeat)

    def schedule(self):
        return smoother_schedule(self.h)

    def close(self):
        if self.h:
            smoother_destroy(self.h)
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
