"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid problems on the host (validation happens
before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2102_00514_amd import binding as B
from paper_2102_00514_amd import workloads as wl

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "smoother.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smoother_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 9
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def test_struct_layout_matches_header():
    # field order of sm_problem in the header
    text = open(HEADER).read()
    body = text[text.index("typedef struct {"):text.index("} sm_problem;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(\w+)\s*[;,]", body)
    assert fields == [f for f, _ in B.sm_problem._fields_]


def test_version_and_defaults():
    assert "gfx950" in B.smoother_version()
    s = B.sm_problem()
    B.lib().smoother_problem_defaults(ctypes.byref(s))
    assert (s.n_tracks, s.n_iter, s.lin, s.precision, s.scan) == (1, 10, 0, 0, 0)
    assert (s.ut_alpha, s.ut_beta, s.ut_kappa) == (1.0, 0.0, 1.0)


def _expect_einval(pb, match, **kw):
    with pytest.raises(B.SmootherError) as ei:
        B.smoother_init(pb, **kw)
    assert ei.value.status == B.SM_EINVAL
    assert re.search(match, str(ei.value)), str(ei.value)


def _c1():
    return wl.config_c1()


def test_rejects_bad_dimensions():
    pb = _c1()
    pb.nx = 7
    _expect_einval(pb, "unsupported")


def test_rejects_bad_offsets():
    pb = _c1()
    pb.offsets = np.array([0, 0], dtype=np.int64)
    _expect_einval(pb, "T >= 1")
    pb = _c1()
    pb.offsets = np.array([1, 100], dtype=np.int64)
    _expect_einval(pb, r"offsets\[0\]")


def test_rejects_non_spd_covariances():
    pb = _c1()
    pb.Q = pb.Q.copy()
    pb.Q[0, 0] = -1.0
    _expect_einval(pb, "Q must be")
    pb = _c1()
    pb.R = np.array([[1.0, 2.0], [2.0, 1.0]])
    _expect_einval(pb, "R must be")
    pb = _c1()
    pb.P0 = pb.P0.copy()
    pb.P0[0, 0, 1] = 0.5     # asymmetric
    _expect_einval(pb, "P0")


def test_rejects_non_finite_measurements():
    pb = _c1()
    pb.y = pb.y.copy()
    pb.y[10, 1] = np.nan
    _expect_einval(pb, "y must be finite")


def test_rejects_bad_params():
    pb = _c1()
    pb.params = pb.params[:-1]
    _expect_einval(pb, "params")
    pb = _c1()
    pb.params = pb.params.copy()
    pb.params[3] = 1.0           # target index 1 does not exist for nx = 5
    _expect_einval(pb, "target")
    pb = _c1()
    pb.params = pb.params.copy()
    pb.params[0] = -0.01
    _expect_einval(pb, "dt")


def test_rejects_bad_options():
    pb = _c1()
    _expect_einval(pb, "unscented", lin="unscented", ut_alpha=1.0, ut_kappa=-5.0)
    _expect_einval(pb, "n_iter", n_iter=-1)
    _expect_einval(pb, "lane_slots", lane_slots=33)
    _expect_einval(pb, "tile_lanes", tile_lanes=100)
    S = pb.n_slots
    _expect_einval(pb, "init_mean", init_mean=np.full((S, 5), np.inf))
    bad_cov = np.tile(np.eye(5), (S, 1, 1))
    bad_cov[3] *= -1
    _expect_einval(pb, "init_cov", init_mean=np.zeros((S, 5)), init_cov=bad_cov)


def test_null_handle_calls_are_state_errors():
    lib = B.lib()
    assert lib.smoother_iterate(None, 1, None, None) == B.SM_ESTATE
    assert lib.smoother_result(None, None, None) == B.SM_ESTATE
    assert lib.smoother_track_deltas(None, None) == B.SM_ESTATE
    assert lib.smoother_objective(None, None) == B.SM_ESTATE
    assert lib.smoother_filter(None, None, None, None) == B.SM_ESTATE
    assert lib.smoother_iterate_lm(None, 1e-2, 10.0, 1e-6, 10, None, None, None) == B.SM_ESTATE
    lib.smoother_destroy(None)   # NULL-safe


WS_HEADER = os.path.join(os.path.dirname(HEADER), "warmstart.h")


def test_warmstart_symbols_and_config_layout():
    from paper_2102_00514_amd import warmstart as W
    text = re.sub(r"/\*.*?\*/", "", open(WS_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(ws_\w+)\s*\(", text)))
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(W.WS_EXPORTS)
    body = text[text.index("typedef struct {"):text.index("} ws_config;")]
    assert re.findall(r"(\w+)\s*;", body) == [f for f, _ in W.ws_config._fields_]
    body = text[text.index("} ws_config;"):text.index("} ws_adam;")]
    body = body[body.index("{") + 1:]
    assert re.findall(r"(\w+)\s*[;,]", body) == [f for f, _ in W.ws_adam._fields_]


def test_warmstart_param_count_and_config_validation():
    from paper_2102_00514_amd import warmstart as W
    from oracle import nn as onn
    assert W.param_count(W.config()) == onn.n_params() == 201876
    for cfgd in (dict(window=16, patch=4, width=16, hidden=2), dict(hidden=0), dict(width=64, hidden=6)):
        c = W.config(**cfgd)
        assert W.param_count(c) == onn.n_params(dict(onn.DEFAULT, **cfgd))
    for bad in (dict(patch=3), dict(window=24, patch=4), dict(hidden=13), dict(max_batch=0), dict(nx=0)):
        c = W.config(**bad)
        assert W.param_count(c) == 0
        h = ctypes.c_void_p()
        st = W._lib.ws_create(ctypes.byref(c), None, ctypes.byref(h))   # validated before any device call
        assert st == W.WS_EINVAL and not h.value
        assert W._lib.ws_last_error(None)


def test_warmstart_null_handles():
    from paper_2102_00514_amd import warmstart as W
    assert W._lib.ws_set_tracks(None, None, 0, None) == W.WS_ESTATE
    assert W._lib.ws_trajectory(None, None, None) == W.WS_ESTATE
    W._lib.ws_destroy(None)
    assert B.lib().smoother_set_trajectory_device(None, None, None, None) == B.SM_ESTATE


def test_one_hip_runtime_in_the_process():
    """The library and PyTorch share a single HIP / HSA runtime (two copies in
    one process leave one of them without a device)."""
    import torch  # noqa: F401
    B.lib()
    maps = open("/proc/self/maps").read().split("\n")
    for name in ("libamdhip64", "libhsa-runtime64"):
        paths = {ln.split()[-1] for ln in maps if name in ln}
        assert len(paths) == 1, (name, paths)


def test_autotune_validates_on_the_host():
    with pytest.raises(B.SmootherError) as ei:
        B.smoother_autotune(wl.config_c1(), iters=2, lin="unscented", ut_kappa=-5.0)
    assert ei.value.status == B.SM_EINVAL
    with pytest.raises(B.SmootherError) as ei:
        B.smoother_autotune(wl.config_c1(), iters=0)
    assert ei.value.status == B.SM_EINVAL


def test_stacked_targets_validation():
    pb = wl.config_c5_single(20)
    bad_q = pb.Q.copy()
    bad_q[0, 7] = bad_q[7, 0] = 1e-6               # couples targets 0 and 1
    pb_q = wl.Problem(**{**pb.__dict__, "Q": bad_q})
    _expect_einval(pb_q, "Q must be block-diagonal")
    bad_r = pb.R.copy()
    bad_r[0, 2] = bad_r[2, 0] = 1e-4                # sensors 0 and 2 watch different targets
    _expect_einval(wl.Problem(**{**pb.__dict__, "R": bad_r}), "R must not couple")
    prm = pb.params.copy()
    prm[3 + 3 * 2] = 0.0                            # three sensors on target 0, one on target 1
    _expect_einval(wl.Problem(**{**pb.__dict__, "params": prm}), "exactly two sensors")
    bad_p0 = pb.P0.copy()
    bad_p0[0, 19, 0] = bad_p0[0, 0, 19] = 0.1
    _expect_einval(wl.Problem(**{**pb.__dict__, "P0": bad_p0}), "P0 must be block-diagonal")


def test_dense_stacked_scope():
    sensors = np.random.default_rng(1).uniform(-2, 2, (6, 2))
    pb3 = wl.stacked_ct(10, np.random.default_rng(2), sensors=sensors, n_targets=3, n_sensors=6)
    _expect_einval(pb3, "unsupported", lin="cubature")                      # only (20, 8) is compiled


def test_rejects_bad_lm_lambda():
    for bad in (-0.5, float("nan"), float("inf")):
        _expect_einval(_c1(), "lm_lambda", lm_lambda=bad)
