"""The engine's FP64 MFMA product for nx = 20 (libdense_probe.so) against the
VALU routine and against numpy: both compute reps * A B for 20 x 20 FP64
matrices; a wrong MFMA operand or result layout gives errors of order one,
rounding about 1e-15 of the result's scale (gate 1e-12).  The phase timer runs
every routine of a combine and reports positive cycle counts."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("blocks,reps", [(1, 1), (7, 3), (300, 2)])
def test_mfma_and_valu_products_match_numpy(blocks, reps):
    import torch
    from paper_2102_00514_amd import dense_probe as dp
    lib = dp.load()
    rng = np.random.default_rng(blocks * 10 + reps)
    A = rng.standard_normal((blocks, 20, 20))
    B = rng.standard_normal((blocks, 20, 20))
    ref = reps * np.einsum("bik,bkj->bij", A, B)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    s = torch.cuda.current_stream().cuda_stream
    for variant in (0, 1):
        C = dp.products(lib, variant, dA, dB, reps, s)
        torch.cuda.synchronize()
        err = np.max(np.abs(C.cpu().numpy() - ref)) / np.max(np.abs(ref))
        assert err < 1e-12, (variant, err)


def test_phase_timer():
    from paper_2102_00514_amd import dense_probe as dp
    for blocks in (1, 3):
        c = dp.phases(blocks, 2)
        assert set(c) == set(dp.PHASES) and all(v > 0 for v in c.values()), c
        # a combine contains two factorisations and ten products
        assert c["filter_combine_eq15"] > 2 * c["cholesky"] + 10 * min(c["product"], c["product_At"]) * 0.5, c
