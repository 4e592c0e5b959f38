"""The allocation-free entry point (smoother_solve_static) against the
allocating one (smoother_init + smoother_iterate + smoother_result_device) on
the same problems, through the C ABI: two calls in a row on the same GPU, the
second with a smaller input, so the second call runs on the scratch the first
one left behind.  Both paths run the same kernels in the same schedule, so the
results agree to the FP64 bar (in practice bit for bit)."""
import numpy as np
import pytest

import oracle
from paper_2102_00514_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32 = 1e-4


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2102_00514_amd import binding
    return binding


def _both(B, pb, M, **kw):
    import torch
    dt = torch.float64 if kw.get("precision", "f64") == "f64" else torch.float32
    S = pb.n_slots
    stream = torch.cuda.current_stream().cuda_stream
    m_ref = torch.empty((S, pb.nx), dtype=dt, device="cuda")
    c_ref = torch.empty((S, pb.nx, pb.nx), dtype=dt, device="cuda")
    with B.Smoother(pb, stream=stream, n_iter=M, lane_slots=1, **kw) as sm:
        d_ref, _ = sm.iterate(0)
        sm.result_device(m_ref.data_ptr(), c_ref.data_ptr())
    m = torch.full((S, pb.nx), float("nan"), dtype=dt, device="cuda")
    c = torch.full((S, pb.nx, pb.nx), float("nan"), dtype=dt, device="cuda")
    torch.cuda.synchronize()
    d = B.smoother_solve_static(pb, m.data_ptr(), c.data_ptr(), stream=stream, n_iter=M, **kw)
    torch.cuda.synchronize()
    return (m.double().cpu().numpy(), c.double().cpu().numpy(), d,
            m_ref.double().cpu().numpy(), c_ref.double().cpu().numpy(), d_ref)


def _check(what, m, c, d, m_ref, c_ref, d_ref, tol):
    em = oracle.mean_error(m, m_ref)
    ep = oracle.cov_error(c, c_ref)
    same = np.array_equal(m, m_ref) and np.array_equal(c, c_ref)
    print(f"{what}: e_m={em:.3e} e_P={ep:.3e} bitwise={same} delta={d:.6e} (allocating path {d_ref:.6e})",
          flush=True)
    assert np.isfinite(m).all() and np.isfinite(c).all()
    assert em <= tol and ep <= tol, (what, em, ep)
    assert abs(d - d_ref) <= 1e-6 * abs(d_ref) + 1e-12


def test_two_calls_second_smaller(B):
    big = wl.config_c2(2 ** 15)               # 32769 slots
    _check("static T=32768 Taylor", *_both(B, big, 3, lin="taylor"), TOL64)
    small = wl.concat_tracks([wl.ct_bearings(T, seed=70 + T) for T in (300, 7, 1, 129)], "ragged")
    _check("static ragged batch cubature", *_both(B, small, 4, lin="cubature", tile_lanes=64), TOL64)


def test_fp32_and_sequential(B):
    pb = wl.config_c1()
    _check("static C1 unscented FP32", *_both(B, pb, 5, lin="unscented", precision="f32"), TOL32)
    _check("static C1 Taylor sequential", *_both(B, pb, 5, lin="taylor", scan="sequential"), TOL64)


def test_limits_are_rejected(B):
    import torch
    pb = wl.ct_bearings(36864, seed=1)        # 36865 slots: one past the maximum
    m = torch.empty((pb.n_slots, 5), dtype=torch.float64, device="cuda")
    c = torch.empty((pb.n_slots, 5, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(B.SmootherError, match="exceeds the static scratch"):
        B.smoother_solve_static(pb, m.data_ptr(), c.data_ptr(), n_iter=1)
    with pytest.raises(B.SmootherError, match="lane_slots"):
        B.smoother_solve_static(wl.config_c1(), m.data_ptr(), c.data_ptr(), n_iter=1, lane_slots=4)
