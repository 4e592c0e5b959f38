"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls it and shares no code with it.

It wraps ``oracle.c``: a plain sequential FP64 (and long double, for
self-checks) iterated extended / sigma-point Kalman filter + RTS smoother, plus
one-at-a-time evaluations of the paper's filtering/smoothing elements and
associative operators (eq. 13-19).  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

LIN = {"taylor": 0, "cubature": 1, "unscented": 2}
ORC_OK, ORC_EINVAL, ORC_ENUMERIC = 0, 1, 4


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile oracle.c twice (double, long double) into liboracle.so."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cflags = ["gcc", "-O2", "-std=c11", "-fPIC", "-Wall", "-Wextra", "-c"]
    objs = []
    # The same source twice: REAL = double and REAL = long double.
    for tag, defs in (("f64", []), ("f80", ["-DORC_LONG"])):
        obj = f"{_LIB_PATH}.{tag}.o"
        subprocess.run(cflags + defs + ["-o", obj, _SRC], check=True)
        objs.append(obj)
    subprocess.run(["gcc", "-shared", "-o", tmp] + objs + ["-lm"], check=True)
    os.replace(tmp, _LIB_PATH)
    for obj in objs:
        os.remove(obj)
    return _LIB_PATH


def build_native(out_dir: str) -> str:
    """Compile oracle.c (double and long double) with -O3 -march=native for the
    host it runs on, into out_dir; for timing the oracle on that host.  The
    portable -O2 build above stays the one the tests load."""
    path = os.path.join(out_dir, "liboracle_native.so")
    objs = []
    for tag, defs in (("f64", []), ("f80", ["-DORC_LONG"])):
        obj = os.path.join(out_dir, f"oracle_native.{tag}.o")
        subprocess.run(["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-c"] + defs + ["-o", obj, _SRC],
                       check=True)
        objs.append(obj)
    subprocess.run(["gcc", "-shared", "-o", path] + objs + ["-lm"], check=True)
    return path


def use_library(path: str) -> None:
    """Route every later call through the oracle library at path (same source,
    other compiler flags)."""
    global _lib
    _lib = ctypes.CDLL(path)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _arr(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _fn(name, prec):
    return getattr(lib(), f"{name}_{prec}")


def _check(rc, what):
    if rc != ORC_OK:
        raise OracleError(f"{what} failed with status {rc}")


def smoother(pb, M: int, lin: str = "taylor", alpha: float = 1.0, beta: float = 0.0,
             kappa: float = 1.0, init_mean=None, init_cov=None, precision: str = "f64",
             history: bool = False, filtered: bool = True, lm_lambda: float = 0.0) -> dict:
    """Iterated smoother on a single-track ``workloads.Problem``.

    lm_lambda > 0: Levenberg-Marquardt damping, each iteration observes the
    previous iterate as a pseudo-measurement with covariance I / lm_lambda.

    Returns mean [T+1, nx], cov [T+1, nx, nx], filt_mean/filt_cov (last
    iteration's filter), deltas [M] and, with ``history``, every iterate."""
    assert pb.n_tracks == 1, "the oracle runs one track at a time"
    nx, ny = pb.nx, pb.ny
    T = int(pb.offsets[1])
    S = T + 1
    out = {"mean": np.empty((S, nx)), "cov": np.empty((S, nx, nx)), "deltas": np.empty(max(M, 1))}
    if filtered:
        out["filt_mean"] = np.empty((S, nx))
        out["filt_cov"] = np.empty((S, nx, nx))
    if history:
        out["hist_mean"] = np.empty((M, S, nx))
        out["hist_cov"] = np.empty((M, S, nx, nx))
    params = _arr(pb.params)
    args = [_arr(pb.Q), _arr(pb.R), _arr(pb.m0[0]), _arr(pb.P0[0]), _arr(pb.y)]
    im = _arr(init_mean, (S, nx)) if init_mean is not None else None
    ic = _arr(init_cov, (S, nx, nx)) if init_cov is not None else None
    rc = _fn("orc_smoother", prec=precision)(
        nx, ny, T, int(pb.model), _ptr(params), int(params.size),
        *[_ptr(a) for a in args], int(M), LIN[lin],
        ctypes.c_double(alpha), ctypes.c_double(beta), ctypes.c_double(kappa),
        _ptr(im), _ptr(ic), _ptr(out["mean"]), _ptr(out["cov"]),
        _ptr(out.get("filt_mean")), _ptr(out.get("filt_cov")),
        _ptr(out.get("hist_mean")), _ptr(out.get("hist_cov")), _ptr(out["deltas"]),
        ctypes.c_double(lm_lambda))
    _check(rc, "orc_smoother")
    out["deltas"] = out["deltas"][:M]
    return out


def smoother_batch(pb, M: int, **kw) -> list:
    """Runs every track of a batch through ``smoother`` (one after the other)."""
    return [smoother(pb.track(i), M, **kw) for i in range(pb.n_tracks)]


def model_eval(pb_or_model, params, nx, ny, x, precision="f64"):
    """f(x), grad f(x), h(x), grad h(x) of a registered model."""
    params = _arr(params)
    x = _arr(x)
    fx, Fx, hx, Hx = np.empty(nx), np.empty((nx, nx)), np.empty(ny), np.empty((ny, nx))
    rc = _fn("orc_model_eval", precision)(int(pb_or_model), _ptr(params), int(params.size), nx, ny,
                                          _ptr(x), _ptr(fx), _ptr(Fx), _ptr(hx), _ptr(Hx))
    _check(rc, "orc_model_eval")
    return fx, Fx, hx, Hx


def sigma_points(mean, cov, lin="cubature", alpha=1.0, beta=0.0, kappa=1.0, precision="f64"):
    mean = _arr(mean)
    n = mean.size
    X = np.empty((2 * n + 1, n))
    w = np.empty(2 * n + 1)
    m = _fn("orc_sigma_points", precision)(n, _ptr(mean), _ptr(_arr(cov)), LIN[lin],
                                           ctypes.c_double(alpha), ctypes.c_double(beta),
                                           ctypes.c_double(kappa), _ptr(X), _ptr(w))
    if m <= 0:
        raise OracleError(f"orc_sigma_points failed with status {-m}")
    return X[:m].copy(), w[:m].copy()


def linearize(model, params, nx, ny, lin, which, xbar, Pbar, alpha=1.0, beta=0.0, kappa=1.0,
              precision="f64"):
    """Linearise f (which='f') or h (which='h') at (xbar, Pbar): (G, g, Lambda)."""
    params = _arr(params)
    q = nx if which == "f" else ny
    G, g, Lam = np.empty((q, nx)), np.empty(q), np.empty((q, q))
    rc = _fn("orc_linearize", precision)(int(model), _ptr(params), int(params.size), nx, ny,
                                         LIN[lin], ctypes.c_double(alpha), ctypes.c_double(beta),
                                         ctypes.c_double(kappa), 0 if which == "f" else 1,
                                         _ptr(_arr(xbar)), _ptr(_arr(Pbar)), _ptr(G), _ptr(g), _ptr(Lam))
    _check(rc, "orc_linearize")
    return G, g, Lam


def linearize_traj(pb, xbar, Pbar, lin="taylor", alpha=1.0, beta=0.0, kappa=1.0, precision="f64"):
    """Surrogate model (eq. 11) of a single track linearised around (xbar, Pbar)."""
    nx, ny, T = pb.nx, pb.ny, int(pb.offsets[1])
    params = _arr(pb.params)
    o = {"F": np.empty((T, nx, nx)), "c": np.empty((T, nx)), "Qp": np.empty((T, nx, nx)),
         "H": np.empty((T, ny, nx)), "d": np.empty((T, ny)), "Rp": np.empty((T, ny, ny)),
         "yt": np.empty((T, ny))}
    rc = _fn("orc_linearize_traj", precision)(
        nx, ny, T, int(pb.model), _ptr(params), int(params.size), _ptr(_arr(pb.Q)), _ptr(_arr(pb.R)),
        _ptr(_arr(pb.y)), LIN[lin], ctypes.c_double(alpha), ctypes.c_double(beta), ctypes.c_double(kappa),
        _ptr(_arr(xbar)), _ptr(_arr(Pbar)), *[_ptr(o[k]) for k in ("F", "c", "Qp", "H", "d", "Rp", "yt")])
    _check(rc, "orc_linearize_traj")
    return o


def kf_rts(lin_model: dict, m0, P0, precision="f64"):
    """One Kalman filter + RTS pass over a surrogate model from ``linearize_traj``."""
    F = _arr(lin_model["F"])
    T, nx = F.shape[0], F.shape[1]
    ny = lin_model["H"].shape[1]
    S = T + 1
    xf, Pf, xs, Ps = np.empty((S, nx)), np.empty((S, nx, nx)), np.empty((S, nx)), np.empty((S, nx, nx))
    rc = _fn("orc_kf_rts", precision)(nx, ny, T, *[_ptr(_arr(lin_model[k])) for k in
                                                   ("F", "c", "Qp", "H", "d", "Rp", "yt")],
                                      _ptr(_arr(m0)), _ptr(_arr(P0)), _ptr(xf), _ptr(Pf), _ptr(xs), _ptr(Ps))
    _check(rc, "orc_kf_rts")
    return {"filt_mean": xf, "filt_cov": Pf, "mean": xs, "cov": Ps}


# --- the paper's building blocks, one at a time -------------------------------------------

def filter_element(F, c, Qp, H, d, Rp, y, precision="f64"):
    """(A, b, C, eta, J) of eq. 13-14, returned packed as [A, b, C, eta, J]."""
    F = _arr(F)
    n, p = F.shape[0], np.asarray(H).shape[0]
    out = np.empty(3 * n * n + 2 * n)
    rc = _fn("orc_filter_element", precision)(n, p, *[_ptr(_arr(a)) for a in (F, c, Qp, H, d, Rp, y)],
                                              _ptr(out))
    _check(rc, "orc_filter_element")
    return out


def filter_combine(ai, aj, n, precision="f64"):
    out = np.empty(3 * n * n + 2 * n)
    rc = _fn("orc_filter_combine", precision)(n, _ptr(_arr(ai)), _ptr(_arr(aj)), _ptr(out))
    _check(rc, "orc_filter_combine")
    return out


def smoother_element(xf, Pf, F, c, Qp, last=False, precision="f64"):
    xf = _arr(xf)
    n = xf.size
    z = np.zeros((n, n))
    out = np.empty(2 * n * n + n)
    rc = _fn("orc_smoother_element", precision)(n, _ptr(xf), _ptr(_arr(Pf)),
                                                _ptr(_arr(F if F is not None else z)),
                                                _ptr(_arr(c if c is not None else np.zeros(n))),
                                                _ptr(_arr(Qp if Qp is not None else z)), int(last), _ptr(out))
    _check(rc, "orc_smoother_element")
    return out


def smoother_combine(ai, aj, n, precision="f64"):
    out = np.empty(2 * n * n + n)
    rc = _fn("orc_smoother_combine", precision)(n, _ptr(_arr(ai)), _ptr(_arr(aj)), _ptr(out))
    _check(rc, "orc_smoother_combine")
    return out


def unpack_filter(e, n):
    nn = n * n
    return (e[:nn].reshape(n, n), e[nn:nn + n], e[nn + n:2 * nn + n].reshape(n, n),
            e[2 * nn + n:2 * nn + 2 * n], e[2 * nn + 2 * n:].reshape(n, n))


def pack_filter(A, b, C, eta, J):
    return np.concatenate([np.ravel(A), np.ravel(b), np.ravel(C), np.ravel(eta), np.ravel(J)])


def unpack_smoother(e, n):
    nn = n * n
    return e[:nn].reshape(n, n), e[nn:nn + n], e[nn + n:].reshape(n, n)


def pack_smoother(E, g, L):
    return np.concatenate([np.ravel(E), np.ravel(g), np.ravel(L)])


# --- parity metrics ----------------------------------------------------------------------

def mean_error(m_test, m_ref, floor=1e-3):
    """max_k ||m_test_k - m_ref_k||_2 / max(||m_ref_k||_2, floor)."""
    d = np.linalg.norm(np.asarray(m_test) - m_ref, axis=-1)
    return float(np.max(d / np.maximum(np.linalg.norm(m_ref, axis=-1), floor)))


def cov_error(P_test, P_ref):
    """max_k ||P_test_k - P_ref_k||_F / ||P_ref_k||_F."""
    d = np.linalg.norm(np.asarray(P_test) - P_ref, axis=(-2, -1))
    return float(np.max(d / np.linalg.norm(P_ref, axis=(-2, -1))))


def map_cost(pb, x, precision: str = "f64") -> float:
    """MAP objective J(x_{0:T}) of a single-track problem (Section 3: the
    function whose Gauss-Newton iterations are the iterated extended smoother):
    prior, transition and measurement residuals weighted by P0^-1, Q^-1, R^-1,
    bearing residuals wrapped to [-pi, pi)."""
    assert pb.n_tracks == 1, "the oracle runs one track at a time"
    nx, ny = pb.nx, pb.ny
    T = int(pb.offsets[1])
    x = _arr(x, (T + 1, nx))
    params = _arr(pb.params)
    out = ctypes.c_double()
    rc = _fn("orc_map_cost", precision)(nx, ny, T, int(pb.model), _ptr(params), int(params.size),
                                         *[_ptr(_arr(a)) for a in (pb.Q, pb.R, pb.m0[0], pb.P0[0], pb.y)],
                                         _ptr(x), ctypes.byref(out))
    _check(rc, "orc_map_cost")
    return out.value


LM_LAMBDA_MAX = 1e16


def lm_adaptive(pb, lam0: float = 1e-2, nu: float = 10.0, tol: float = 1e-6, max_iter: int = 50,
                accept_rtol: float = 1e-12, init_mean=None, init_cov=None, stop: bool = True) -> dict:
    """Levenberg-Marquardt iterated extended smoother with Marquardt's damping
    schedule, one track.

    Every iteration is one damped pass (``smoother(..., M=1, lm_lambda=lam)``)
    from the current iterate.  The step is taken when it does not raise the MAP
    objective by more than accept_rtol |J| (rounding of J), and then lam /= nu;
    otherwise the iterate is kept and lam = min(lam * nu, LM_LAMBDA_MAX).  The
    track has converged at the first taken step whose largest change is below
    tol while lam (the value the step used) is at most lam0.  With ``stop`` the
    loop ends there, otherwise it runs max_iter iterations.

    Returns mean, cov, first (1-based iteration of convergence, 0 if none),
    iters, and per iteration: lam (used), cost (after the decision), taken,
    delta (of the damped pass), cost_new (of the damped pass's result)."""
    nx = pb.nx
    T = int(pb.offsets[1])
    S = T + 1
    xb = np.broadcast_to(pb.m0[0], (S, nx)).copy() if init_mean is None else _arr(init_mean, (S, nx)).copy()
    Pb = np.broadcast_to(pb.P0[0], (S, nx, nx)).copy() if init_cov is None else _arr(init_cov, (S, nx, nx)).copy()
    J = map_cost(pb, xb)
    lam = lam0
    hist = {"lam": [], "cost": [], "taken": [], "delta": [], "cost_new": []}
    first = 0
    it = 0
    while it < max_iter:
        it += 1
        r = smoother(pb, 1, "taylor", init_mean=xb, init_cov=Pb, lm_lambda=lam, filtered=False)
        Jn = map_cost(pb, r["mean"])
        d = float(r["deltas"][0])
        taken = bool(Jn <= J + accept_rtol * abs(J))
        hist["lam"].append(lam)
        hist["delta"].append(d)
        hist["cost_new"].append(Jn)
        hist["taken"].append(taken)
        if taken:
            if first == 0 and d < tol and lam <= lam0:
                first = it
            xb, Pb, J = r["mean"], r["cov"], Jn
            lam = lam / nu
        else:
            lam = min(lam * nu, LM_LAMBDA_MAX)
        hist["cost"].append(J)
        if stop and first:
            break
    out = {"mean": xb, "cov": Pb, "first": first, "iters": it, "final_cost": J}
    out.update({k: np.array(v) for k, v in hist.items()})
    return out


def filter_loglik(pb, lin: str = "taylor", alpha: float = 1.0, beta: float = 0.0, kappa: float = 1.0,
                  init_mean=None, init_cov=None, precision: str = "f64") -> dict:
    """One filtering pass of a single track linearised at (init_mean, init_cov)
    (default: the prior broadcast): filt_mean [T+1, nx], filt_cov [T+1, nx, nx]
    and loglik = log p(y_{1:T}) of the linearised model, the sum of the
    Gaussian predictive log densities."""
    assert pb.n_tracks == 1, "the oracle runs one track at a time"
    nx, ny = pb.nx, pb.ny
    T = int(pb.offsets[1])
    S = T + 1
    out = {"filt_mean": np.empty((S, nx)), "filt_cov": np.empty((S, nx, nx))}
    params = _arr(pb.params)
    im = _arr(init_mean, (S, nx)) if init_mean is not None else None
    ic = _arr(init_cov, (S, nx, nx)) if init_cov is not None else None
    ll = ctypes.c_double()
    rc = _fn("orc_filter_loglik", precision)(
        nx, ny, T, int(pb.model), _ptr(params), int(params.size),
        *[_ptr(_arr(a)) for a in (pb.Q, pb.R, pb.m0[0], pb.P0[0], pb.y)], LIN[lin],
        ctypes.c_double(alpha), ctypes.c_double(beta), ctypes.c_double(kappa),
        _ptr(im), _ptr(ic), _ptr(out["filt_mean"]), _ptr(out["filt_cov"]), ctypes.byref(ll))
    _check(rc, "orc_filter_loglik")
    out["loglik"] = ll.value
    return out
