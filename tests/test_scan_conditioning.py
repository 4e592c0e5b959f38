"""Rounding of the parallel filtering scan itself (CPU, oracle building blocks).

The first iteration of C3 track 0 (T = 6667, prior turn rate 0, P0 = I,
cubature) is the case where the GPU's parallel scan and the sequential oracle
differ by 2e-9 to 7e-9 (by schedule).  This test shows that the gap belongs to the method in FP64,
not to the kernels: the paper's filtering operator (eq. 15, as the oracle
evaluates it) applied in a Kogge-Stone order in FP64 differs from the 80-bit
sequential Kalman/RTS result by more than 1e-9, while the FP64 sequential
recursion stays within 1e-10, and the smoothing scan (eq. 19) in the same
order is accurate when it starts from accurate filtered moments.

The second test bounds the FP32 variants the same way: with every combine exact,
FP32 storage of the scans' operands alone sets the error floor at long tracks.
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


def _r32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def _via_fp32_factor(M, n):
    """M = Z Z^T rebuilt from its symmetric factor Z rounded to FP32."""
    M = M.reshape(n, n)
    if not np.any(M):
        return M.ravel()
    w, V = np.linalg.eigh(0.5 * (M + M.T))
    Z = _r32(V * np.sqrt(np.maximum(w, 0.0)))
    return (Z @ Z.T).ravel()


def test_fp32_storage_bounds_an_fp32_tree_scan():
    """What an FP32 parallel smoother can reach at all: operands stored in FP32.

    Iteration 5 of T = 4096 (IEKS, from the oracle's iterate 4).  Two FP32
    effects, each with the rest exact (FP64):
    - the surrogate model, trajectory and prior rounded to FP32, then the
      sequential recursion: ~5e-7 on the smoothed covariances;
    - the eq. 15 / eq. 19 scans in Kogge-Stone order with every element and
      every combined result rounded to FP32 (each combine itself exact):
      ~7e-6, once with C, J, L rounded as they are and once through FP32
      factors (the square-root form's storage).
    Storage rounding inside the tree-order scan costs more than ten times what
    rounding the linearisation's inputs and outputs costs, and factor storage
    does not remove it: at T = 2^15 both storages give 2e-5 (cubature) to 3e-5
    (IEKS) on their own, so an FP32 scan in this order cannot reach 1e-5 at
    that length, whatever the element form."""
    T = 4096
    pb = wl.config_c2(T)
    n, nn = pb.nx, pb.nx * pb.nx
    ref = oracle.smoother(pb, 5, "taylor", history=True)
    xb, Pb = ref["hist_mean"][3], ref["hist_cov"][3]
    lm = oracle.linearize_traj(pb, xb, Pb, "taylor")
    exact = oracle.kf_rts(lm, pb.m0[0], pb.P0[0])
    assert oracle.cov_error(exact["cov"], ref["hist_cov"][4]) < 1e-12

    lm32 = {k: _r32(v) for k, v in oracle.linearize_traj(pb, _r32(xb), _r32(Pb), "taylor").items()}
    seq = oracle.kf_rts(lm32, _r32(pb.m0[0]), _r32(pb.P0[0]))
    e_model = oracle.cov_error(seq["cov"], exact["cov"])

    def round_plain(e):
        return _r32(e)

    def round_filter_factored(e):
        e = e.copy()
        for s in (slice(0, nn), slice(nn, nn + n), slice(2 * nn + n, 2 * nn + 2 * n)):
            e[s] = _r32(e[s])
        e[nn + n:2 * nn + n] = _via_fp32_factor(e[nn + n:2 * nn + n], n)
        e[2 * nn + 2 * n:] = _via_fp32_factor(e[2 * nn + 2 * n:], n)
        return e

    def round_smoother_factored(e):
        e = e.copy()
        e[:nn + n] = _r32(e[:nn + n])
        e[nn + n:] = _via_fp32_factor(e[nn + n:], n)
        return e

    fe = [oracle.pack_filter(np.zeros((n, n)), pb.m0[0], pb.P0[0], np.zeros(n), np.zeros((n, n)))]
    for k in range(T):
        fe.append(oracle.filter_element(lm["F"][k], lm["c"][k], lm["Qp"][k], lm["H"][k], lm["d"][k],
                                        lm["Rp"][k], lm["yt"][k]))
    errs = {}
    for name, rf, rs in (("plain", round_plain, round_plain),
                         ("factored", round_filter_factored, round_smoother_factored)):
        pref = kogge_stone([rf(e) for e in fe], lambda a, b: rf(oracle.filter_combine(a, b, n)))
        xf = np.array([oracle.unpack_filter(e, n)[1] for e in pref])
        Pf = np.array([oracle.unpack_filter(e, n)[2] for e in pref])
        se = [oracle.smoother_element(xf[k], Pf[k], lm["F"][k], lm["c"][k], lm["Qp"][k]) for k in range(T)]
        se.append(oracle.smoother_element(xf[T], Pf[T], None, None, None, last=True))
        suf = kogge_stone([rs(e) for e in se[::-1]], lambda a, b: rs(oracle.smoother_combine(b, a, n)))[::-1]
        Ps = np.array([oracle.unpack_smoother(e, n)[2] for e in suf])
        errs[name] = oracle.cov_error(Ps, exact["cov"])
    print(f"T={T} smoothed e_P: model in FP32 {e_model:.2e}; FP32 scan storage plain {errs['plain']:.2e}, "
          f"factored {errs['factored']:.2e}")
    assert e_model < 1.5e-6
    for name, e in errs.items():
        assert e > 3e-6 and e > 5 * e_model, (name, e, e_model)
