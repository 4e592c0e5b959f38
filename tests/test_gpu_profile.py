"""smoother_profile_repeat: the profiling pass launches every kernel several
times back to back between one pair of HIP events.  Each kernel of an
iteration computes its outputs from buffers it does not write and the
per-track change statistic is a maximum, so the trajectory and the deltas
after profiled iterations must equal, bit for bit, those after the same
number of ordinary iterations.  Checked on every engine path."""
import numpy as np
import pytest

from paper_2102_00514_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2102_00514_amd import binding
    return binding


def _ragged():
    return wl.concat_tracks([wl.ct_bearings(T, seed=90 + T) for T in (300, 7, 1, 1200, 40)], "ragged")


CASES = [
    ("c1 taylor", lambda: wl.config_c1(), dict(lin="taylor")),
    ("ragged cubature 64x8", _ragged, dict(lin="cubature", tile_lanes=64, lane_slots=8)),
    ("ragged unscented 256x2", _ragged, dict(lin="unscented", tile_lanes=256, lane_slots=2)),
    ("sequential scan", _ragged, dict(lin="cubature", scan="sequential")),
    ("sqrt form", _ragged, dict(lin="taylor", form="sqrt", lane_slots=4)),
    ("fp32", lambda: wl.config_c1(), dict(lin="cubature", precision="f32")),
    ("nx=20 unscented", lambda: wl.config_c5_single(300), dict(lin="unscented")),
    ("stacked taylor blocks", lambda: wl.stacked_ct(300, np.random.default_rng([57, 300])), dict(lin="taylor")),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_profiled_iterations_equal_ordinary_ones(B, name, make, kw):
    pb = make()
    with B.Smoother(pb, n_iter=3, **kw) as sm:
        sm.iterate(1, want_delta=False)
        prof = sm.profile(2, repeat=4)
        m_p, c_p = sm.result()
        d_p = sm.track_deltas()
    with B.Smoother(pb, n_iter=3, **kw) as sm:
        sm.iterate(3, want_delta=False)
        m_i, c_i = sm.result()
        d_i = sm.track_deltas()
    assert prof and all(v[0] > 0 and v[1] > 0 for v in prof.values()), prof
    assert np.array_equal(m_p, m_i) and np.array_equal(c_p, c_i), name
    assert np.array_equal(d_p, d_i, equal_nan=True), (name, d_p, d_i)


def test_repeat_outside_range_is_rejected(B):
    with B.Smoother(wl.config_c1()) as sm:
        for bad in (0, 65):
            with pytest.raises(B.SmootherError, match="repeat"):
                sm.profile(1, repeat=bad)
