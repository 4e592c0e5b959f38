"""Independent references used to pin the oracle (tests only).

Nothing here reuses the oracle's arithmetic:
  * the coordinated-turn transition is obtained by integrating its ODE
    (px' = vx, py' = vy, vx' = -w vy, vy' = w vx, w' = 0) with classical RK4;
  * Jacobians come from complex-step differentiation of these functions;
  * bearings use numpy's arctan2 for values and complex arctan for slopes;
  * posteriors and Gauss-Newton steps are dense least-squares solves over the
    whole trajectory x_{0:T} (no recursion).
"""
from __future__ import annotations

import numpy as np

CS_H = 1e-30  # complex-step size


def ct_ode_step(x, dt, substeps=256):
    """Coordinated-turn transition of stacked 5-blocks by RK4 on the ODE.

    Works for complex inputs (complex-step differentiation)."""
    x = np.asarray(x)
    nb = x.shape[-1] // 5

    def rhs(z):
        out = np.zeros_like(z)
        for b in range(nb):
            o = 5 * b
            vx, vy, w = z[..., o + 2], z[..., o + 3], z[..., o + 4]
            out[..., o] = vx
            out[..., o + 1] = vy
            out[..., o + 2] = -w * vy
            out[..., o + 3] = w * vx
        return out

    h = dt / substeps
    z = x.astype(np.result_type(x.dtype, np.float64))
    for _ in range(substeps):
        k1 = rhs(z)
        k2 = rhs(z + 0.5 * h * k1)
        k3 = rhs(z + 0.5 * h * k2)
        k4 = rhs(z + h * k3)
        z = z + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return z


def _atan2_cs(dy, dx):
    """atan2 whose imaginary part carries the complex-step derivative."""
    val = np.arctan2(np.real(dy), np.real(dx))
    if not np.iscomplexobj(dy) and not np.iscomplexobj(dx):
        return val
    dy = np.asarray(dy, dtype=complex)
    dx = np.asarray(dx, dtype=complex)
    use_x = np.abs(np.real(dx)) >= np.abs(np.real(dy))
    with np.errstate(all="ignore"):
        s1 = np.arctan(dy / np.where(use_x, dx, 1.0))          # atan2 = atan(dy/dx) + const
        s2 = -np.arctan(dx / np.where(use_x, 1.0, dy))         # atan2 = -atan(dx/dy) + const
    slope = np.where(use_x, np.imag(s1), np.imag(s2))
    return val + 1j * slope


def bearings(x, sensors, targets):
    x = np.asarray(x)
    out = []
    for (sx, sy), t in zip(sensors, targets):
        t = int(t)
        out.append(_atan2_cs(x[..., 5 * t + 1] - sy, x[..., 5 * t] - sx))
    return np.stack(out, axis=-1)


def cs_jacobian(fun, x):
    """Complex-step Jacobian of fun: R^n -> R^m at x."""
    x = np.asarray(x, dtype=np.float64)
    cols = []
    for j in range(x.size):
        xc = x.astype(complex)
        xc[j] += 1j * CS_H
        cols.append(np.imag(fun(xc)) / CS_H)
    return np.stack(cols, axis=-1)


def wrap(a):
    return a - 2.0 * np.pi * np.floor((a + np.pi) / (2.0 * np.pi))


def ct_model_funcs(pb):
    """(f, h) of a MODEL_CT_BEARINGS problem built from the ODE and arctan2."""
    dt = pb.params[0]
    blk = pb.params[1:].reshape(-1, 3)
    sensors, targets = blk[:, :2], blk[:, 2]
    return (lambda x: ct_ode_step(x, dt)), (lambda x: bearings(x, sensors, targets))


def linear_model_funcs(pb):
    n, p = pb.nx, pb.ny
    prm = pb.params
    F = prm[:n * n].reshape(n, n)
    c = prm[n * n:n * n + n]
    H = prm[n * n + n:n * n + n + p * n].reshape(p, n)
    d = prm[n * n + n + p * n:]
    return (lambda x: x @ F.T + c), (lambda x: x @ H.T + d)


def map_residual(pb, f, h, angular):
    """Whitened residual r(x_{0:T}) of the MAP objective
       1/2 |x0-m0|^2_{P0^-1} + 1/2 sum |x_k - f(x_{k-1})|^2_{Q^-1}
       + 1/2 sum |y_k - h(x_k)|^2_{R^-1}   (bearing residuals wrapped)."""
    n = pb.nx
    T = int(pb.offsets[1])
    W0 = np.linalg.inv(np.linalg.cholesky(pb.P0[0]))
    Wq = np.linalg.inv(np.linalg.cholesky(pb.Q))
    Wr = np.linalg.inv(np.linalg.cholesky(pb.R))
    m0, y = pb.m0[0], pb.y

    def r(xflat):
        X = xflat.reshape(T + 1, n)
        r0 = (X[0] - m0) @ W0.T
        rq = (X[1:] - f(X[:-1])) @ Wq.T
        hv = h(X[1:])
        if angular:
            # wrap the value, keep the complex-step slope of -h
            e = wrap(np.real(y - hv)) + 1j * np.imag(-hv) if np.iscomplexobj(hv) else wrap(y - hv)
        else:
            e = y - hv
        rr = e @ Wr.T
        return np.concatenate([r0.ravel(), rq.ravel(), rr.ravel()])

    return r


def gauss_newton(pb, f, h, angular, x_init, iters, lam=0.0):
    """Dense Gauss-Newton on the MAP objective over x_{0:T}; with lam > 0 each
    step is Levenberg-Marquardt damped: the rows sqrt(lam) (x - x_lin) are
    appended to the linearised residual.

    Returns the list of iterates and, for each step, the marginal covariances
    (diagonal blocks of (J^T J + lam I)^-1 at the linearisation point)."""
    n = pb.nx
    T = int(pb.offsets[1])
    r = map_residual(pb, f, h, angular)
    x = np.asarray(x_init, dtype=np.float64).ravel().copy()
    xs, covs = [], []
    for _ in range(iters):
        J = cs_jacobian(r, x)
        res = r(x)
        if lam > 0:
            J = np.vstack([J, np.sqrt(lam) * np.eye(x.size)])
            res = np.concatenate([res, np.zeros(x.size)])
        step, *_ = np.linalg.lstsq(J, -res, rcond=None)
        x = x + step
        Qf, Rf = np.linalg.qr(J)
        Rinv = np.linalg.inv(Rf)
        cov = Rinv @ Rinv.T
        xs.append(x.reshape(T + 1, n).copy())
        covs.append(np.stack([cov[k * n:(k + 1) * n, k * n:(k + 1) * n] for k in range(T + 1)]))
    return xs, covs


def dense_linear_posterior(pb):
    """Exact posterior of x_{0:T} for an affine-Gaussian model by one dense
    least-squares solve (means) and the inverse normal matrix (covariances)."""
    f, h = linear_model_funcs(pb)
    n = pb.nx
    T = int(pb.offsets[1])
    xs, covs = gauss_newton(pb, f, h, False, np.zeros((T + 1, n)), 1)
    return xs[0], covs[0]


def gaussian_cubic_expectation(mu, P, a, B, Cc):
    """E[g(x)], x ~ N(mu, P), g(x) = a.x + x^T B x + sum C_ijk x_i x_j x_k."""
    e1 = a @ mu
    e2 = np.einsum("ij,ij->", B, np.outer(mu, mu) + P)
    m3 = (np.einsum("i,j,k->ijk", mu, mu, mu) + np.einsum("i,jk->ijk", mu, P)
          + np.einsum("j,ik->ijk", mu, P) + np.einsum("k,ij->ijk", mu, P))
    e3 = np.einsum("ijk,ijk->", Cc, m3)
    return e1 + e2 + e3
