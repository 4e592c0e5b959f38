"""Rounding of the parallel filtering scan itself (CPU, oracle building blocks).

The first iteration of C3 track 0 (T = 6667, prior turn rate 0, P0 = I,
cubature) is the case where the GPU's parallel scan and the sequential oracle
differ by 2.2e-9.  This test shows that the gap belongs to the method in FP64,
not to the kernels: the paper's filtering operator (eq. 15, as the oracle
evaluates it) applied in a Kogge-Stone order in FP64 differs from the 80-bit
sequential Kalman/RTS result by more than 1e-9, while the FP64 sequential
recursion stays within 1e-10, and the smoothing scan (eq. 19) in the same
order is accurate when it starts from accurate filtered moments.
"""
import numpy as np

import oracle
from paper_2102_00514_amd import workloads as wl


def kogge_stone(elems, op):
    cur, d = list(elems), 1
    while d < len(cur):
        cur = [cur[i] if i < d else op(cur[i - d], cur[i]) for i in range(len(cur))]
        d *= 2
    return cur


def test_tree_order_filtering_scan_is_ill_conditioned_on_c3_track_0():
    pb = wl.ct_batch(1, 100, 8192, seed_tag=3)       # track 0 of the C3 batch
    T, n = int(pb.offsets[1]), pb.nx
    assert T == 6667
    xb = np.repeat(pb.m0, T + 1, axis=0)
    Pb = np.repeat(pb.P0, T + 1, axis=0)
    lm = oracle.linearize_traj(pb, xb, Pb, "cubature")
    lm80 = oracle.linearize_traj(pb, xb, Pb, "cubature", precision="f80")
    ref = oracle.kf_rts(lm80, pb.m0[0], pb.P0[0], precision="f80")
    seq = oracle.kf_rts(lm, pb.m0[0], pb.P0[0])
    assert oracle.mean_error(seq["mean"], ref["mean"]) < 1e-10
    assert oracle.cov_error(seq["cov"], ref["cov"]) < 1e-10

    # filtering elements (slot 0: prior element) and their tree-ordered prefix
    elems = [oracle.pack_filter(np.zeros((n, n)), pb.m0[0], pb.P0[0], np.zeros(n), np.zeros((n, n)))]
    for k in range(T):
        elems.append(oracle.filter_element(lm["F"][k], lm["c"][k], lm["Qp"][k], lm["H"][k], lm["d"][k],
                                           lm["Rp"][k], lm["yt"][k]))
    pref = kogge_stone(elems, lambda a, b: oracle.filter_combine(a, b, n))
    xf = np.array([oracle.unpack_filter(e, n)[1] for e in pref])
    Pf = np.array([oracle.unpack_filter(e, n)[2] for e in pref])
    em = oracle.mean_error(xf, ref["filt_mean"])
    print(f"Kogge-Stone filtering scan, FP64: e_m={em:.2e}; sequential FP64 filter: "
          f"{oracle.mean_error(seq['filt_mean'], ref['filt_mean']):.2e}")
    assert em > 1e-9

    # the smoothing scan in the same order, from the 80-bit filtered moments
    se = [oracle.smoother_element(ref["filt_mean"][k], ref["filt_cov"][k], lm["F"][k], lm["c"][k], lm["Qp"][k])
          for k in range(T)]
    se.append(oracle.smoother_element(ref["filt_mean"][T], ref["filt_cov"][T], None, None, None, last=True))
    suf = kogge_stone(se[::-1], lambda a, b: oracle.smoother_combine(b, a, n))[::-1]
    xs = np.array([oracle.unpack_smoother(e, n)[1] for e in suf])
    Ps = np.array([oracle.unpack_smoother(e, n)[2] for e in suf])
    assert oracle.mean_error(xs, ref["mean"]) < 1e-10
    assert oracle.cov_error(Ps, ref["cov"]) < 1e-10
