/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call,
 * link or load this file; it is used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark.
 *
 * A plain, sequential, obviously-correct CPU reference for the iterated
 * extended (Taylor) and sigma-point (statistical linear regression) Kalman
 * smoothers of Yaghoobi, Corenflos, Hassan and Sarkka, "Parallel Iterated
 * Extended and Sigma-Point Kalman Smoothers" (ICASSP 2021).
 *
 * The parallel method of the paper reaches, for every iteration, exactly the
 * result of the sequential Kalman filter and Rauch-Tung-Striebel smoother run on
 * that iteration's linearised model (Section 2: the filter is the prefix of the
 * filtering elements and the smoother the suffix of the smoothing elements).
 * The oracle is therefore that sequential definition:
 *
 *   repeat M times (Section 3, iterated smoothers):
 *     1. linearise f at every slot k = 0..T-1 and h at k = 1..T around the
 *        previous smoothed trajectory (xbar_k, Pbar_k):
 *          Taylor:  F = grad f(xbar), c = f(xbar) - F xbar, Lambda = 0   (eq. 10)
 *                   H = grad h(xbar), d = h(xbar) - H xbar, Omega = 0
 *          SLR:     sigma points of (xbar, Pbar), moments zbar, Psi, Phi (eq. 8),
 *                   F = Psi^T Pbar^-1, c = zbar - F xbar,
 *                   Lambda = Phi - F Pbar F^T                          (eq. 7, 9)
 *     2. Kalman filter on the surrogate x_k = F x_{k-1} + c + N(0, Q + Lambda),
 *        y_k = H x_k + d + N(0, R + Omega) (eq. 11) from (m0, P0);
 *     3. RTS smoother back to slot 0.
 *
 * It also evaluates, one by one, the paper's parallel building blocks -- the
 * filtering element (eq. 13-14), the filtering operator (eq. 15), the smoothing
 * element (eq. 16-18) and the smoothing operator (eq. 19) -- so that tests can
 * check the identities that tie them to the sequential definition.
 *
 * Readings of the paper taken here (each is a test-visible convention):
 *   - the state x_0 is part of the smoothed trajectory and F_0 is linearised at
 *     the smoothed xbar_0 (the problem asks for the posterior of x_{0:n});
 *   - the offsets of eq. 13 and 14 use d_k (the printed d_{k-1} in b_k is a typo),
 *     and eta_k has no trailing H_k (dimensions);
 *   - the smoothing gain is E_k = P*_k F_k^T (F_k P*_k F_k^T + Q'_k)^-1;
 *   - the first iteration starts from the prior broadcast over all slots unless
 *     an initial trajectory is given;
 *   - cubature points are xbar +- sqrt(n) L e_j with L the lower Cholesky factor
 *     of Pbar and weights 1/(2n); unscented points use lambda = alpha^2 (n+kappa) - n,
 *     spread sqrt(n+lambda), weights lambda/(n+lambda) and 1/(2(n+lambda)), one
 *     weight set for means and covariances (beta is accepted and unused);
 *   - bearing outputs are unwrapped around h(xbar_k): the measurement becomes
 *     h(xbar_k) + wrap(y_k - h(xbar_k)) and each sigma image
 *     h(xbar_k) + wrap(h(X_j) - h(xbar_k)), with wrap mapping to [-pi, pi);
 *   - stored covariances are symmetrised, (P + P^T)/2.
 *
 * The file is compiled twice: with REAL = double (exported names end in _f64)
 * and with REAL = long double (names end in _f80), so that a test can measure
 * the oracle's own rounding error.  Every exported function takes and returns
 * double arrays; long double is internal only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORC_LONG
typedef double real;
#define SFX(name) name##_f64
#define RSIN sin
#define RCOS cos
#define RSQRT sqrt
#define RATAN2 atan2
#define RFLOOR floor
#define RFABS fabs
#define RLOG log
#define RPI 3.14159265358979323846264338327950288
#else
typedef long double real;
#define SFX(name) name##_f80
#define RSIN sinl
#define RCOS cosl
#define RSQRT sqrtl
#define RATAN2 atan2l
#define RFLOOR floorl
#define RFABS fabsl
#define RLOG logl
#define RPI 3.14159265358979323846264338327950288L
#endif

#define NMAX 32          /* largest state / measurement dimension handled */
#define SMAX (2 * NMAX + 1)

enum { MODEL_LINEAR = 0, MODEL_CT_BEARINGS = 1 };
enum { LIN_TAYLOR = 0, LIN_CUBATURE = 1, LIN_UNSCENTED = 2 };
enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENUMERIC = 4 };

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra, row-major, dimensions <= NMAX.                  */
/* ------------------------------------------------------------------------ */

/* C (m x n) = A (m x k) B (k x n) */
static void mm(int m, int k, int n, const real *A, const real *B, real *C) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            real s = 0;
            for (int t = 0; t < k; ++t) s += A[i * k + t] * B[t * n + j];
            C[i * n + j] = s;
        }
}

/* C (m x n) = A (m x k) B^T, B is (n x k) */
static void mmt(int m, int k, int n, const real *A, const real *B, real *C) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            real s = 0;
            for (int t = 0; t < k; ++t) s += A[i * k + t] * B[j * k + t];
            C[i * n + j] = s;
        }
}

/* C (m x n) = A^T B, A is (k x m), B is (k x n) */
static void mtm(int m, int k, int n, const real *A, const real *B, real *C) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            real s = 0;
            for (int t = 0; t < k; ++t) s += A[t * m + i] * B[t * n + j];
            C[i * n + j] = s;
        }
}

/* y (m) = A (m x n) x */
static void mv(int m, int n, const real *A, const real *x, real *y) {
    for (int i = 0; i < m; ++i) {
        real s = 0;
        for (int t = 0; t < n; ++t) s += A[i * n + t] * x[t];
        y[i] = s;
    }
}

static void symmetrize(int n, real *A) {
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            real s = (A[i * n + j] + A[j * n + i]) / 2;
            A[i * n + j] = s;
            A[j * n + i] = s;
        }
}

/* Lower Cholesky factor L of a symmetric positive-definite A (A = L L^T).
 * Returns 0, or -1 if A is not numerically positive definite. */
static int chol(int n, const real *A, real *L) {
    memset(L, 0, sizeof(real) * n * n);
    for (int j = 0; j < n; ++j) {
        real s = A[j * n + j];
        for (int t = 0; t < j; ++t) s -= L[j * n + t] * L[j * n + t];
        if (!(s > 0)) return -1;
        real d = RSQRT(s);
        L[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            real v = A[i * n + j];
            for (int t = 0; t < j; ++t) v -= L[i * n + t] * L[j * n + t];
            L[i * n + j] = v / d;
        }
    }
    return 0;
}

/* Solve (L L^T) X = B in place, B is (n x nrhs). */
static void chol_solve(int n, const real *L, real *B, int nrhs) {
    for (int r = 0; r < nrhs; ++r) {
        for (int i = 0; i < n; ++i) {          /* L z = b */
            real s = B[i * nrhs + r];
            for (int t = 0; t < i; ++t) s -= L[i * n + t] * B[t * nrhs + r];
            B[i * nrhs + r] = s / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {     /* L^T x = z */
            real s = B[i * nrhs + r];
            for (int t = i + 1; t < n; ++t) s -= L[t * n + i] * B[t * nrhs + r];
            B[i * nrhs + r] = s / L[i * n + i];
        }
    }
}

/* Solve A X = B (A general, n x n) by Gaussian elimination with partial
 * pivoting; A and B are overwritten.  Returns -1 on an exactly singular pivot. */
static int gauss_solve(int n, real *A, real *B, int nrhs) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (RFABS(A[i * n + k]) > RFABS(A[p * n + k])) p = i;
        if (A[p * n + k] == 0) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) { real t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
            for (int j = 0; j < nrhs; ++j) { real t = B[k * nrhs + j]; B[k * nrhs + j] = B[p * nrhs + j]; B[p * nrhs + j] = t; }
        }
        for (int i = k + 1; i < n; ++i) {
            real l = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
            for (int j = 0; j < nrhs; ++j) B[i * nrhs + j] -= l * B[k * nrhs + j];
        }
    }
    for (int i = n - 1; i >= 0; --i)
        for (int j = 0; j < nrhs; ++j) {
            real s = B[i * nrhs + j];
            for (int t = i + 1; t < n; ++t) s -= A[i * n + t] * B[t * nrhs + j];
            B[i * nrhs + j] = s / A[i * n + i];
        }
    return 0;
}

static void load(real *dst, const double *src, int n) { for (int i = 0; i < n; ++i) dst[i] = (real)src[i]; }
static void store(double *dst, const real *src, int n) { for (int i = 0; i < n; ++i) dst[i] = (double)src[i]; }

static real wrap_angle(real a) { return a - 2 * RPI * RFLOOR((a + RPI) / (2 * RPI)); }

/* ------------------------------------------------------------------------ */
/* Models (the f and h of the additive-noise state-space model, eq. 4).        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int model, nx, ny, n_params;
    real p[NMAX * NMAX + 2 * NMAX + NMAX * NMAX + NMAX + 1];
} model_t;

static int model_setup(model_t *md, int model, const double *params, int n_params, int nx, int ny) {
    if (nx < 1 || ny < 1 || nx > NMAX || ny > NMAX) return ORC_EINVAL;
    md->model = model; md->nx = nx; md->ny = ny; md->n_params = n_params;
    if (model == MODEL_LINEAR) {
        if (n_params != nx * nx + nx + ny * nx + ny) return ORC_EINVAL;
    } else if (model == MODEL_CT_BEARINGS) {
        if (nx % 5 != 0 || n_params != 1 + 3 * ny) return ORC_EINVAL;
        for (int s = 0; s < ny; ++s) {
            double t = params[1 + 3 * s + 2];
            if (t < 0 || t >= nx / 5 || t != (int)t) return ORC_EINVAL;
        }
    } else {
        return ORC_EINVAL;
    }
    if (n_params > (int)(sizeof(md->p) / sizeof(md->p[0]))) return ORC_EINVAL;
    load(md->p, params, n_params);
    return ORC_OK;
}

/* Coordinated-turn coefficients for a = omega*dt:
 *   s1 = sin(a)/omega, s2 = (1 - cos a)/omega and their omega-derivatives.
 * A truncated Taylor series is used for |a| < 0.1 (it also covers omega = 0). */
static void ct_coeffs(real w, real dt, real *s1, real *s2, real *ds1, real *ds2) {
    real a = w * dt;
    if (RFABS(a) < (real)0.1) {
        real a2 = a * a;
        *s1 = dt * (1 - a2 / 6 * (1 - a2 / 20 * (1 - a2 / 42 * (1 - a2 / 72))));
        *s2 = dt * a * ((real)1 / 2 - a2 / 24 * (1 - a2 / 30 * (1 - a2 / 56 * (1 - a2 / 90))));
        *ds1 = dt * dt * (-a / 3 + a * a2 / 30 - a * a2 * a2 / 840 + a * a2 * a2 * a2 / 45360
                          - a * a2 * a2 * a2 * a2 / 3991680);
        *ds2 = dt * dt * ((real)1 / 2 - a2 / 8 + a2 * a2 / 144 - a2 * a2 * a2 / 5760
                          + a2 * a2 * a2 * a2 / 403200);
    } else {
        real sa = RSIN(a), ca = RCOS(a), hs = RSIN(a / 2);
        real omc = 2 * hs * hs;                       /* 1 - cos a */
        *s1 = sa / w;
        *s2 = omc / w;
        *ds1 = dt * dt * (a * ca - sa) / (a * a);
        *ds2 = dt * dt * (a * sa - omc) / (a * a);
    }
}

/* fx = f(x); if Fx is not NULL also the Jacobian (nx x nx). */
static void model_f(const model_t *md, const real *x, real *fx, real *Fx) {
    int n = md->nx;
    if (md->model == MODEL_LINEAR) {
        const real *F = md->p, *c = md->p + n * n;
        mv(n, n, F, x, fx);
        for (int i = 0; i < n; ++i) fx[i] += c[i];
        if (Fx) memcpy(Fx, F, sizeof(real) * n * n);
        return;
    }
    real dt = md->p[0];
    if (Fx) memset(Fx, 0, sizeof(real) * n * n);
    for (int b = 0; b < n / 5; ++b) {
        const real *xb = x + 5 * b;
        real *fb = fx + 5 * b;
        real vx = xb[2], vy = xb[3], w = xb[4];
        real s1, s2, ds1, ds2;
        ct_coeffs(w, dt, &s1, &s2, &ds1, &ds2);
        real a = w * dt, sa = RSIN(a), ca = RCOS(a);
        fb[0] = xb[0] + s1 * vx - s2 * vy;
        fb[1] = xb[1] + s2 * vx + s1 * vy;
        fb[2] = ca * vx - sa * vy;
        fb[3] = sa * vx + ca * vy;
        fb[4] = w;
        if (Fx) {
            int o = 5 * b;
#define J(i, j) Fx[(o + (i)) * n + o + (j)]
            J(0, 0) = 1; J(0, 2) = s1; J(0, 3) = -s2; J(0, 4) = ds1 * vx - ds2 * vy;
            J(1, 1) = 1; J(1, 2) = s2; J(1, 3) = s1;  J(1, 4) = ds2 * vx + ds1 * vy;
            J(2, 2) = ca; J(2, 3) = -sa; J(2, 4) = -dt * (sa * vx + ca * vy);
            J(3, 2) = sa; J(3, 3) = ca;  J(3, 4) = dt * (ca * vx - sa * vy);
            J(4, 4) = 1;
#undef J
        }
    }
}

/* hx = h(x); if Hx is not NULL also the Jacobian (ny x nx). */
static void model_h(const model_t *md, const real *x, real *hx, real *Hx) {
    int n = md->nx, p = md->ny;
    if (md->model == MODEL_LINEAR) {
        const real *H = md->p + n * n + n, *d = H + p * n;
        mv(p, n, H, x, hx);
        for (int i = 0; i < p; ++i) hx[i] += d[i];
        if (Hx) memcpy(Hx, H, sizeof(real) * p * n);
        return;
    }
    if (Hx) memset(Hx, 0, sizeof(real) * p * n);
    for (int s = 0; s < p; ++s) {
        real sx = md->p[1 + 3 * s], sy = md->p[2 + 3 * s];
        int t = (int)md->p[3 + 3 * s];
        real dx = x[5 * t] - sx, dy = x[5 * t + 1] - sy;
        hx[s] = RATAN2(dy, dx);
        if (Hx) {
            real r2 = dx * dx + dy * dy;
            Hx[s * n + 5 * t] = -dy / r2;
            Hx[s * n + 5 * t + 1] = dx / r2;
        }
    }
}

static int model_angular_y(const model_t *md) { return md->model == MODEL_CT_BEARINGS; }

/* ------------------------------------------------------------------------ */
/* Sigma points (Section 3, iterated sigma-point method).                      */
/* ------------------------------------------------------------------------ */


/* Points X (m x n) and weights w (m) for N(mean, cov).  Returns m, or -1 if cov
 * is not positive definite. */
static int sigma_points(int n, const real *mean, const real *cov, int lin, real alpha, real kappa,
                        real *X, real *w) {
    real L[NMAX * NMAX];
    if (chol(n, cov, L)) return -1;
    real spread, w0 = 0, wj;
    int off;
    if (lin == LIN_CUBATURE) {
        spread = RSQRT((real)n);
        wj = (real)1 / (2 * n);
        off = 0;
    } else {
        real lam = alpha * alpha * (n + kappa) - n;
        spread = RSQRT(n + lam);
        w0 = lam / (n + lam);
        wj = 1 / (2 * (n + lam));
        off = 1;
        for (int i = 0; i < n; ++i) X[i] = mean[i];
        w[0] = w0;
    }
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            X[(off + j) * n + i] = mean[i] + spread * L[i * n + j];
            X[(off + n + j) * n + i] = mean[i] - spread * L[i * n + j];
        }
        w[off + j] = wj;
        w[off + n + j] = wj;
    }
    return off + 2 * n;
}

/* ------------------------------------------------------------------------ */
/* Linearisation of one function at one slot.                                */
/* which = 0: f (n -> n), which = 1: h (n -> p).                               */
/* Outputs the affine map G x + g and the extra noise Lam (eq. 5).             */
/* For h of an angular model, href = h(xbar) is also returned (unwrap centre). */
/* ------------------------------------------------------------------------ */

static int linearize_one(const model_t *md, int which, int lin, real alpha, real kappa,
                         const real *xbar, const real *Pbar, real *G, real *g, real *Lam, real *href) {
    int n = md->nx, q = which ? md->ny : md->nx;
    int ang = which && model_angular_y(md);
    real z0[NMAX];
    if (which) model_h(md, xbar, z0, lin == LIN_TAYLOR ? G : NULL);
    else model_f(md, xbar, z0, lin == LIN_TAYLOR ? G : NULL);
    if (href) memcpy(href, z0, sizeof(real) * q);
    if (lin == LIN_TAYLOR) {
        /* eq. 10: G = Jacobian, g = f(xbar) - G xbar, no extra noise. */
        real Gx[NMAX];
        mv(q, n, G, xbar, Gx);
        for (int i = 0; i < q; ++i) g[i] = z0[i] - Gx[i];
        memset(Lam, 0, sizeof(real) * q * q);
        return ORC_OK;
    }
    /* eq. 7-9: statistical linear regression with sigma points. */
    real X[SMAX * NMAX], w[SMAX], Z[SMAX * NMAX];
    int m = sigma_points(n, xbar, Pbar, lin, alpha, kappa, X, w);
    if (m < 0) return ORC_ENUMERIC;
    for (int j = 0; j < m; ++j) {
        if (which) model_h(md, X + j * n, Z + j * q, NULL);
        else model_f(md, X + j * n, Z + j * q, NULL);
        if (ang)
            for (int i = 0; i < q; ++i) Z[j * q + i] = z0[i] + wrap_angle(Z[j * q + i] - z0[i]);
    }
    real zbar[NMAX] = {0}, Psi[NMAX * NMAX] = {0}, Phi[NMAX * NMAX] = {0};
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < q; ++i) zbar[i] += w[j] * Z[j * q + i];
    for (int j = 0; j < m; ++j)
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < q; ++b)
                Psi[a * q + b] += w[j] * (X[j * n + a] - xbar[a]) * (Z[j * q + b] - zbar[b]);
    for (int j = 0; j < m; ++j)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                Phi[a * q + b] += w[j] * (Z[j * q + a] - zbar[a]) * (Z[j * q + b] - zbar[b]);
    /* G = Psi^T Pbar^-1, i.e. Pbar G^T = Psi. */
    real L[NMAX * NMAX], Gt[NMAX * NMAX];
    if (chol(n, Pbar, L)) return ORC_ENUMERIC;
    memcpy(Gt, Psi, sizeof(real) * n * q);
    chol_solve(n, L, Gt, q);
    for (int i = 0; i < q; ++i)
        for (int a = 0; a < n; ++a) G[i * n + a] = Gt[a * q + i];
    real Gx[NMAX];
    mv(q, n, G, xbar, Gx);
    for (int i = 0; i < q; ++i) g[i] = zbar[i] - Gx[i];
    /* Lam = Phi - G Pbar G^T */
    real GP[NMAX * NMAX], GPG[NMAX * NMAX];
    mm(q, n, n, G, Pbar, GP);
    mmt(q, n, q, GP, G, GPG);
    for (int i = 0; i < q * q; ++i) Lam[i] = Phi[i] - GPG[i];
    symmetrize(q, Lam);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One linearised pass: Kalman filter + RTS smoother over slots 0..T.         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, p, T;
    real *F, *c, *Qp;     /* slots 0..T-1: F_k, c_k, Q'_k = Q + Lambda_k */
    real *H, *d, *Rp;     /* slots 1..T (index k-1): H_k, d_k, R'_k = R + Omega_k */
    real *yt;             /* slots 1..T (index k-1): unwrapped measurement */
} linpass_t;

/*
 * Levenberg-Marquardt damping of the Gauss-Newton step (Section 3 remark on
 * IEKS as Gauss-Newton and its Levenberg-Marquardt extension): the previous
 * iterate xbar_k is observed as a pseudo-measurement z = x_k + v,
 * v ~ N(0, I / lam), which adds (lam / 2) |x_k - xbar_k|^2 to the MAP
 * objective of every slot.  Kalman update of (m, P) with H = I, R = I / lam.
 */
static int lm_update(int n, real *m, real *P, const real *z, real lam) {
    real S[NMAX * NMAX], L[NMAX * NMAX], Kt[NMAX * NMAX], KP[NMAX * NMAX];
    memcpy(S, P, sizeof(real) * n * n);
    for (int i = 0; i < n; ++i) S[i * n + i] += 1 / lam;
    if (chol(n, S, L)) return ORC_ENUMERIC;
    memcpy(Kt, P, sizeof(real) * n * n);          /* K^T = S^-1 P (P symmetric) */
    chol_solve(n, L, Kt, n);
    real e[NMAX];
    for (int i = 0; i < n; ++i) e[i] = z[i] - m[i];
    for (int i = 0; i < n; ++i) {
        real s = m[i];
        for (int j = 0; j < n; ++j) s += Kt[j * n + i] * e[j];
        m[i] = s;
    }
    mtm(n, n, n, Kt, P, KP);                      /* K P = (S^-1 P)^T P */
    for (int i = 0; i < n * n; ++i) P[i] -= KP[i];
    symmetrize(n, P);
    return ORC_OK;
}

static int kf_rts(const linpass_t *lp, const real *m0, const real *P0, real lam, const real *xbar,
                  real *xf, real *Pf, real *xs, real *Ps) {
    int n = lp->n, p = lp->p, T = lp->T;
    memcpy(xf, m0, sizeof(real) * n);
    memcpy(Pf, P0, sizeof(real) * n * n);
    if (lam > 0 && lm_update(n, xf, Pf, xbar, lam)) return ORC_ENUMERIC;
    real mp[NMAX], Pp[NMAX * NMAX], tmp[NMAX * NMAX], S[NMAX * NMAX], L[NMAX * NMAX];
    real PHt[NMAX * NMAX], K[NMAX * NMAX], v[NMAX], Hm[NMAX], KS[NMAX * NMAX], KSK[NMAX * NMAX];
    for (int k = 1; k <= T; ++k) {
        const real *F = lp->F + (k - 1) * n * n, *c = lp->c + (k - 1) * n, *Qp = lp->Qp + (k - 1) * n * n;
        const real *H = lp->H + (k - 1) * p * n, *d = lp->d + (k - 1) * p, *Rp = lp->Rp + (k - 1) * p * p;
        const real *yk = lp->yt + (k - 1) * p;
        const real *m = xf + (k - 1) * n, *P = Pf + (k - 1) * n * n;
        /* predict */
        mv(n, n, F, m, mp);
        for (int i = 0; i < n; ++i) mp[i] += c[i];
        mm(n, n, n, F, P, tmp);
        mmt(n, n, n, tmp, F, Pp);
        for (int i = 0; i < n * n; ++i) Pp[i] += Qp[i];
        symmetrize(n, Pp);
        /* update */
        mmt(n, n, p, Pp, H, PHt);                 /* P- H^T (n x p) */
        mm(p, n, p, H, PHt, S);                   /* H P- H^T */
        for (int i = 0; i < p * p; ++i) S[i] += Rp[i];
        symmetrize(p, S);
        if (chol(p, S, L)) return ORC_ENUMERIC;
        for (int i = 0; i < n; ++i)               /* K^T = S^-1 (P- H^T)^T */
            for (int j = 0; j < p; ++j) K[j * n + i] = PHt[i * p + j];
        chol_solve(p, L, K, n);                   /* K holds K^T (p x n) */
        mv(p, n, H, mp, Hm);
        for (int j = 0; j < p; ++j) v[j] = yk[j] - Hm[j] - d[j];
        real *mk = xf + k * n, *Pk = Pf + k * n * n;
        for (int i = 0; i < n; ++i) {
            real s = mp[i];
            for (int j = 0; j < p; ++j) s += K[j * n + i] * v[j];
            mk[i] = s;
        }
        mtm(n, p, p, K, S, KS);                   /* K S (n x p) */
        mm(n, p, n, KS, K, KSK);                  /* K S K^T */
        for (int i = 0; i < n * n; ++i) Pk[i] = Pp[i] - KSK[i];
        symmetrize(n, Pk);
        if (lam > 0 && lm_update(n, mk, Pk, xbar + k * n, lam)) return ORC_ENUMERIC;
    }
    memcpy(xs + T * n, xf + T * n, sizeof(real) * n);
    memcpy(Ps + T * n * n, Pf + T * n * n, sizeof(real) * n * n);
    real G[NMAX * NMAX], Gt[NMAX * NMAX], dm[NMAX], dP[NMAX * NMAX], Gd[NMAX * NMAX];
    for (int k = T - 1; k >= 0; --k) {
        const real *F = lp->F + k * n * n, *c = lp->c + k * n, *Qp = lp->Qp + k * n * n;
        const real *m = xf + k * n, *P = Pf + k * n * n;
        mm(n, n, n, F, P, tmp);                   /* F P* */
        mmt(n, n, n, tmp, F, Pp);                 /* F P* F^T */
        for (int i = 0; i < n * n; ++i) Pp[i] += Qp[i];
        symmetrize(n, Pp);
        if (chol(n, Pp, L)) return ORC_ENUMERIC;
        memcpy(Gt, tmp, sizeof(real) * n * n);    /* G^T = (P-)^-1 F P* */
        chol_solve(n, L, Gt, n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) G[i * n + j] = Gt[j * n + i];
        mv(n, n, F, m, mp);
        for (int i = 0; i < n; ++i) dm[i] = xs[(k + 1) * n + i] - mp[i] - c[i];
        for (int i = 0; i < n; ++i) {
            real s = m[i];
            for (int j = 0; j < n; ++j) s += G[i * n + j] * dm[j];
            xs[k * n + i] = s;
        }
        for (int i = 0; i < n * n; ++i) dP[i] = Ps[(k + 1) * n * n + i] - Pp[i];
        mm(n, n, n, G, dP, Gd);
        mmt(n, n, n, Gd, G, tmp);
        for (int i = 0; i < n * n; ++i) Ps[k * n * n + i] = P[i] + tmp[i];
        symmetrize(n, Ps + k * n * n);
    }
    return ORC_OK;
}

static int linpass_alloc(linpass_t *lp, int n, int p, int T) {
    lp->n = n; lp->p = p; lp->T = T;
    size_t Tn = (size_t)(T > 0 ? T : 1);
    lp->F = malloc(sizeof(real) * Tn * n * n);
    lp->c = malloc(sizeof(real) * Tn * n);
    lp->Qp = malloc(sizeof(real) * Tn * n * n);
    lp->H = malloc(sizeof(real) * Tn * p * n);
    lp->d = malloc(sizeof(real) * Tn * p);
    lp->Rp = malloc(sizeof(real) * Tn * p * p);
    lp->yt = malloc(sizeof(real) * Tn * p);
    return (lp->F && lp->c && lp->Qp && lp->H && lp->d && lp->Rp && lp->yt) ? ORC_OK : -1;
}

static void linpass_free(linpass_t *lp) {
    free(lp->F); free(lp->c); free(lp->Qp); free(lp->H); free(lp->d); free(lp->Rp); free(lp->yt);
}

/* Linearise the whole trajectory (xbar, Pbar over slots 0..T). */
static int linearize_traj(const model_t *md, int lin, real alpha, real kappa, const real *Q, const real *R,
                          const real *y, const real *xbar, const real *Pbar, linpass_t *lp) {
    int n = md->nx, p = md->ny, T = lp->T;
    real Lam[NMAX * NMAX], href[NMAX];
    for (int k = 0; k < T; ++k) {
        int rc = linearize_one(md, 0, lin, alpha, kappa, xbar + k * n, Pbar + k * n * n,
                               lp->F + k * n * n, lp->c + k * n, Lam, NULL);
        if (rc) return rc;
        for (int i = 0; i < n * n; ++i) lp->Qp[k * n * n + i] = Q[i] + Lam[i];
    }
    for (int k = 1; k <= T; ++k) {
        int rc = linearize_one(md, 1, lin, alpha, kappa, xbar + k * n, Pbar + k * n * n,
                               lp->H + (k - 1) * p * n, lp->d + (k - 1) * p, Lam, href);
        if (rc) return rc;
        for (int i = 0; i < p * p; ++i) lp->Rp[(k - 1) * p * p + i] = R[i] + Lam[i];
        for (int i = 0; i < p; ++i) {
            real yk = y[(k - 1) * p + i];
            lp->yt[(k - 1) * p + i] = model_angular_y(md) ? href[i] + wrap_angle(yk - href[i]) : yk;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exported: the iterated smoother (single track).                            */
/* ------------------------------------------------------------------------ */

/*
 * Runs M iterations of the iterated smoother on one track with T measurements.
 *   y [T][ny]; Q [nx][nx]; R [ny][ny]; m0 [nx]; P0 [nx][nx];
 *   init_mean [T+1][nx], init_cov [T+1][nx][nx] (both NULL = prior broadcast);
 * Outputs (NULL to skip):
 *   mean [T+1][nx], cov [T+1][nx][nx]     smoothed result of the last iteration;
 *   filt_mean, filt_cov (same shapes)     filtered result of the last iteration;
 *   hist_mean [M][T+1][nx], hist_cov [M][T+1][nx][nx]  every iterate;
 *   deltas [M]   max_k,j |xbar^(i) - xbar^(i-1)|.
 * lm_lambda > 0 damps every iteration by the pseudo-measurement of lm_update.
 * Returns 0, 1 (invalid argument) or 4 (a Cholesky factorisation failed).
 */
int SFX(orc_smoother)(int nx, int ny, int T, int model, const double *params, int n_params,
                      const double *Q, const double *R, const double *m0, const double *P0,
                      const double *y, int M, int lin, double alpha, double beta, double kappa,
                      const double *init_mean, const double *init_cov,
                      double *mean, double *cov, double *filt_mean, double *filt_cov,
                      double *hist_mean, double *hist_cov, double *deltas, double lm_lambda) {
    (void)beta;
    model_t md;
    if (T < 0 || M < 0 || lin < 0 || lin > 2 || !(lm_lambda >= 0)) return ORC_EINVAL;
    int rc = model_setup(&md, model, params, n_params, nx, ny);
    if (rc) return rc;
    int n = nx, p = ny;
    size_t S = (size_t)T + 1;
    real *xb = malloc(sizeof(real) * S * n), *Pb = malloc(sizeof(real) * S * n * n);
    real *xf = malloc(sizeof(real) * S * n), *Pf = malloc(sizeof(real) * S * n * n);
    real *xs = malloc(sizeof(real) * S * n), *Ps = malloc(sizeof(real) * S * n * n);
    real *yy = malloc(sizeof(real) * (T > 0 ? T : 1) * p);
    real Qr[NMAX * NMAX], Rr[NMAX * NMAX], m0r[NMAX], P0r[NMAX * NMAX];
    linpass_t lp;
    rc = linpass_alloc(&lp, n, p, T);
    if (rc || !xb || !Pb || !xf || !Pf || !xs || !Ps || !yy) { rc = ORC_EINVAL; goto done; }
    load(Qr, Q, n * n); load(Rr, R, p * p); load(m0r, m0, n); load(P0r, P0, n * n);
    load(yy, y, T * p);
    if (init_mean) load(xb, init_mean, (int)(S * n));
    else for (size_t k = 0; k < S; ++k) memcpy(xb + k * n, m0r, sizeof(real) * n);
    if (init_cov) load(Pb, init_cov, (int)(S * n * n));
    else for (size_t k = 0; k < S; ++k) memcpy(Pb + k * n * n, P0r, sizeof(real) * n * n);
    if (M == 0) {
        memcpy(xs, xb, sizeof(real) * S * n);
        memcpy(Ps, Pb, sizeof(real) * S * n * n);
        memset(xf, 0, sizeof(real) * S * n);
        memset(Pf, 0, sizeof(real) * S * n * n);
    }
    for (int it = 0; it < M; ++it) {
        rc = linearize_traj(&md, lin, (real)alpha, (real)kappa, Qr, Rr, yy, xb, Pb, &lp);
        if (rc) goto done;
        rc = kf_rts(&lp, m0r, P0r, (real)lm_lambda, xb, xf, Pf, xs, Ps);
        if (rc) goto done;
        real dmax = 0;
        for (size_t i = 0; i < S * n; ++i) {
            real dlt = RFABS(xs[i] - xb[i]);
            if (!(dlt <= dmax)) dmax = dlt;         /* NaN propagates */
        }
        if (deltas) deltas[it] = (double)dmax;
        if (hist_mean) store(hist_mean + (size_t)it * S * n, xs, (int)(S * n));
        if (hist_cov) store(hist_cov + (size_t)it * S * n * n, Ps, (int)(S * n * n));
        memcpy(xb, xs, sizeof(real) * S * n);
        memcpy(Pb, Ps, sizeof(real) * S * n * n);
    }
    if (mean) store(mean, xs, (int)(S * n));
    if (cov) store(cov, Ps, (int)(S * n * n));
    if (filt_mean) store(filt_mean, xf, (int)(S * n));
    if (filt_cov) store(filt_cov, Pf, (int)(S * n * n));
    rc = ORC_OK;
done:
    linpass_free(&lp);
    free(xb); free(Pb); free(xf); free(Pf); free(xs); free(Ps); free(yy);
    return rc;
}

/*
 * Kalman filter of one linearised pass with the log marginal likelihood of the
 * surrogate model (Section 2: the filtering prefix a_1 (x) ... (x) a_k carries
 * p(x_k | y_{1:k}) and, with the normalising constants, p(y_{1:k})).  By the
 * chain rule p(y_{1:T}) = prod_k p(y_k | y_{1:k-1}), and each factor is the
 * Gaussian predictive density N(y_k; H_k m-_k + d_k, H_k P-_k H_k^T + R'_k).
 */
static int kf_loglik(const linpass_t *lp, const real *m0, const real *P0, real *xf, real *Pf, real *loglik) {
    int n = lp->n, p = lp->p, T = lp->T;
    memcpy(xf, m0, sizeof(real) * n);
    memcpy(Pf, P0, sizeof(real) * n * n);
    real ll = 0;
    real mp[NMAX], Pp[NMAX * NMAX], tmp[NMAX * NMAX], S[NMAX * NMAX], L[NMAX * NMAX];
    real PHt[NMAX * NMAX], K[NMAX * NMAX], v[NMAX], w[NMAX], Hm[NMAX], KS[NMAX * NMAX], KSK[NMAX * NMAX];
    for (int k = 1; k <= T; ++k) {
        const real *F = lp->F + (k - 1) * n * n, *c = lp->c + (k - 1) * n, *Qp = lp->Qp + (k - 1) * n * n;
        const real *H = lp->H + (k - 1) * p * n, *d = lp->d + (k - 1) * p, *Rp = lp->Rp + (k - 1) * p * p;
        const real *yk = lp->yt + (k - 1) * p;
        const real *m = xf + (k - 1) * n, *P = Pf + (k - 1) * n * n;
        mv(n, n, F, m, mp);
        for (int i = 0; i < n; ++i) mp[i] += c[i];
        mm(n, n, n, F, P, tmp);
        mmt(n, n, n, tmp, F, Pp);
        for (int i = 0; i < n * n; ++i) Pp[i] += Qp[i];
        symmetrize(n, Pp);
        mmt(n, n, p, Pp, H, PHt);
        mm(p, n, p, H, PHt, S);
        for (int i = 0; i < p * p; ++i) S[i] += Rp[i];
        symmetrize(p, S);
        if (chol(p, S, L)) return ORC_ENUMERIC;
        mv(p, n, H, mp, Hm);
        for (int j = 0; j < p; ++j) v[j] = yk[j] - Hm[j] - d[j];
        /* log N(v; 0, S) = -1/2 (p log 2 pi + log det S + v^T S^-1 v) */
        memcpy(w, v, sizeof(real) * p);
        chol_solve(p, L, w, 1);
        real quad = 0, logdet = 0;
        for (int j = 0; j < p; ++j) {
            quad += v[j] * w[j];
            logdet += 2 * RLOG(L[j * p + j]);
        }
        ll -= (p * RLOG(2 * RPI) + logdet + quad) / 2;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < p; ++j) K[j * n + i] = PHt[i * p + j];
        chol_solve(p, L, K, n);
        real *mk = xf + k * n, *Pk = Pf + k * n * n;
        for (int i = 0; i < n; ++i) {
            real s = mp[i];
            for (int j = 0; j < p; ++j) s += K[j * n + i] * v[j];
            mk[i] = s;
        }
        mtm(n, p, p, K, S, KS);
        mm(n, p, n, KS, K, KSK);
        for (int i = 0; i < n * n; ++i) Pk[i] = Pp[i] - KSK[i];
        symmetrize(n, Pk);
    }
    *loglik = ll;
    return ORC_OK;
}

/*
 * One filtering pass linearised at (xbar, Pbar) over slots 0..T (both NULL =
 * prior broadcast, as the first iteration of orc_smoother): filtered means
 * filt_mean [T+1][nx] and covariances filt_cov [T+1][nx][nx] (nullable) and
 * *loglik = log p(y_{1:T}) of the linearised model (for a linear model, the
 * exact marginal likelihood).
 */
int SFX(orc_filter_loglik)(int nx, int ny, int T, int model, const double *params, int n_params,
                           const double *Q, const double *R, const double *m0, const double *P0,
                           const double *y, int lin, double alpha, double beta, double kappa,
                           const double *xbar, const double *Pbar, double *filt_mean, double *filt_cov,
                           double *loglik) {
    (void)beta;
    model_t md;
    if (T < 0 || lin < 0 || lin > 2 || !loglik) return ORC_EINVAL;
    int rc = model_setup(&md, model, params, n_params, nx, ny);
    if (rc) return rc;
    int n = nx, p = ny;
    size_t S = (size_t)T + 1;
    real *xb = malloc(sizeof(real) * S * n), *Pb = malloc(sizeof(real) * S * n * n);
    real *xf = malloc(sizeof(real) * S * n), *Pf = malloc(sizeof(real) * S * n * n);
    real *yy = malloc(sizeof(real) * (T > 0 ? T : 1) * p);
    real Qr[NMAX * NMAX], Rr[NMAX * NMAX], m0r[NMAX], P0r[NMAX * NMAX], ll = 0;
    linpass_t lp;
    rc = linpass_alloc(&lp, n, p, T);
    if (rc || !xb || !Pb || !xf || !Pf || !yy) { rc = ORC_EINVAL; goto done; }
    load(Qr, Q, n * n); load(Rr, R, p * p); load(m0r, m0, n); load(P0r, P0, n * n);
    load(yy, y, T * p);
    if (xbar) load(xb, xbar, (int)(S * n));
    else for (size_t k = 0; k < S; ++k) memcpy(xb + k * n, m0r, sizeof(real) * n);
    if (Pbar) load(Pb, Pbar, (int)(S * n * n));
    else for (size_t k = 0; k < S; ++k) memcpy(Pb + k * n * n, P0r, sizeof(real) * n * n);
    rc = linearize_traj(&md, lin, (real)alpha, (real)kappa, Qr, Rr, yy, xb, Pb, &lp);
    if (rc) goto done;
    rc = kf_loglik(&lp, m0r, P0r, xf, Pf, &ll);
    if (rc) goto done;
    if (filt_mean) store(filt_mean, xf, (int)(S * n));
    if (filt_cov) store(filt_cov, Pf, (int)(S * n * n));
    *loglik = (double)ll;
    rc = ORC_OK;
done:
    linpass_free(&lp);
    free(xb); free(Pb); free(xf); free(Pf); free(yy);
    return rc;
}

/*
 * MAP objective of the trajectory x = x_{0:T} (Section 3: the iterated
 * extended smoother is Gauss-Newton on it, and its Levenberg-Marquardt
 * extension decides on it whether a damped step is taken):
 *   J(x) = 1/2 |x_0 - m0|^2_{P0^-1}
 *        + sum_{k=1..T} 1/2 |x_k - f(x_{k-1})|^2_{Q^-1} + 1/2 |y_k - h(x_k)|^2_{R^-1},
 * with |v|^2_{A^-1} = v^T A^-1 v.  For bearing measurements the residual
 * y_k - h(x_k) is taken modulo 2 pi in [-pi, pi), the same unwrapping the
 * linearisation uses.  x is [T+1][nx]; *cost receives J.
 * Returns 0, 1 (invalid argument) or 4 (P0, Q or R not positive definite).
 */
int SFX(orc_map_cost)(int nx, int ny, int T, int model, const double *params, int n_params,
                      const double *Q, const double *R, const double *m0, const double *P0,
                      const double *y, const double *x, double *cost) {
    model_t md;
    if (T < 0 || !x || !cost) return ORC_EINVAL;
    int rc = model_setup(&md, model, params, n_params, nx, ny);
    if (rc) return rc;
    int n = nx, p = ny;
    real A[NMAX * NMAX], LQ[NMAX * NMAX], LR[NMAX * NMAX], L0[NMAX * NMAX];
    load(A, Q, n * n);
    if (chol(n, A, LQ)) return ORC_ENUMERIC;
    load(A, R, p * p);
    if (chol(p, A, LR)) return ORC_ENUMERIC;
    load(A, P0, n * n);
    if (chol(n, A, L0)) return ORC_ENUMERIC;
    real xp[NMAX], xk[NMAX], fx[NMAX], hx[NMAX], r[NMAX], z[NMAX];
    real total = 0;
    load(xk, x, n);
    for (int i = 0; i < n; ++i) r[i] = xk[i] - (real)m0[i];
    memcpy(z, r, sizeof(real) * n);
    chol_solve(n, L0, z, 1);
    for (int i = 0; i < n; ++i) total += r[i] * z[i] / 2;
    for (int k = 1; k <= T; ++k) {
        memcpy(xp, xk, sizeof(real) * n);
        load(xk, x + (size_t)k * n, n);
        model_f(&md, xp, fx, NULL);
        for (int i = 0; i < n; ++i) r[i] = xk[i] - fx[i];
        memcpy(z, r, sizeof(real) * n);
        chol_solve(n, LQ, z, 1);
        for (int i = 0; i < n; ++i) total += r[i] * z[i] / 2;
        model_h(&md, xk, hx, NULL);
        for (int i = 0; i < p; ++i) {
            r[i] = (real)y[(size_t)(k - 1) * p + i] - hx[i];
            if (model_angular_y(&md)) r[i] = wrap_angle(r[i]);
        }
        memcpy(z, r, sizeof(real) * p);
        chol_solve(p, LR, z, 1);
        for (int i = 0; i < p; ++i) total += r[i] * z[i] / 2;
    }
    *cost = (double)total;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exported: model evaluation, sigma points, single-slot linearisation.        */
/* ------------------------------------------------------------------------ */

/* fx [nx], Fx [nx][nx] (nullable); hx [ny], Hx [ny][nx] (nullable). */
int SFX(orc_model_eval)(int model, const double *params, int n_params, int nx, int ny,
                        const double *x, double *fx, double *Fx, double *hx, double *Hx) {
    model_t md;
    int rc = model_setup(&md, model, params, n_params, nx, ny);
    if (rc) return rc;
    real xr[NMAX], f[NMAX], Fr[NMAX * NMAX], h[NMAX], Hr[NMAX * NMAX];
    load(xr, x, nx);
    model_f(&md, xr, f, Fx ? Fr : NULL);
    model_h(&md, xr, h, Hx ? Hr : NULL);
    if (fx) store(fx, f, nx);
    if (Fx) store(Fx, Fr, nx * nx);
    if (hx) store(hx, h, ny);
    if (Hx) store(Hx, Hr, ny * nx);
    return ORC_OK;
}

/* X [m][n], w [m]; returns m (> 0) or -4 if cov is not positive definite. */
int SFX(orc_sigma_points)(int n, const double *mean, const double *cov, int lin,
                          double alpha, double beta, double kappa, double *X, double *w) {
    (void)beta;
    if (n < 1 || n > NMAX || lin < 1 || lin > 2) return -ORC_EINVAL;
    real mr[NMAX], cr[NMAX * NMAX], Xr[SMAX * NMAX], wr[SMAX];
    load(mr, mean, n); load(cr, cov, n * n);
    int m = sigma_points(n, mr, cr, lin, (real)alpha, (real)kappa, Xr, wr);
    if (m < 0) return -ORC_ENUMERIC;
    store(X, Xr, m * n); store(w, wr, m);
    return m;
}

/* Linearise f (which = 0) or h (which = 1) at (xbar, Pbar):
 * G [q][nx], g [q], Lam [q][q] with q = nx or ny. */
int SFX(orc_linearize)(int model, const double *params, int n_params, int nx, int ny, int lin,
                       double alpha, double beta, double kappa, int which,
                       const double *xbar, const double *Pbar, double *G, double *g, double *Lam) {
    (void)beta;
    model_t md;
    int rc = model_setup(&md, model, params, n_params, nx, ny);
    if (rc) return rc;
    int q = which ? ny : nx;
    real xr[NMAX], Pr[NMAX * NMAX], Gr[NMAX * NMAX], gr[NMAX], Lr[NMAX * NMAX];
    load(xr, xbar, nx); load(Pr, Pbar, nx * nx);
    rc = linearize_one(&md, which, lin, (real)alpha, (real)kappa, xr, Pr, Gr, gr, Lr, NULL);
    if (rc) return rc;
    store(G, Gr, q * nx); store(g, gr, q); store(Lam, Lr, q * q);
    return ORC_OK;
}

/*
 * Linearise a whole trajectory (slots 0..T) and return the surrogate model
 * of eq. 11: F [T][nx][nx], c [T][nx], Qp [T][nx][nx] for slots 0..T-1 and
 * H [T][ny][nx], d [T][ny], Rp [T][ny][ny], yt [T][ny] for slots 1..T.
 */
int SFX(orc_linearize_traj)(int nx, int ny, int T, int model, const double *params, int n_params,
                            const double *Q, const double *R, const double *y, int lin,
                            double alpha, double beta, double kappa,
                            const double *xbar, const double *Pbar,
                            double *F, double *c, double *Qp, double *H, double *d, double *Rp, double *yt) {
    (void)beta;
    model_t md;
    int rc = model_setup(&md, model, params, n_params, nx, ny);
    if (rc) return rc;
    int n = nx, p = ny;
    size_t S = (size_t)T + 1;
    linpass_t lp;
    real *xb = malloc(sizeof(real) * S * n), *Pb = malloc(sizeof(real) * S * n * n);
    real *yy = malloc(sizeof(real) * (T > 0 ? T : 1) * p);
    real Qr[NMAX * NMAX], Rr[NMAX * NMAX];
    rc = linpass_alloc(&lp, n, p, T);
    if (rc || !xb || !Pb || !yy) { rc = ORC_EINVAL; goto done; }
    load(Qr, Q, n * n); load(Rr, R, p * p); load(yy, y, T * p);
    load(xb, xbar, (int)(S * n)); load(Pb, Pbar, (int)(S * n * n));
    rc = linearize_traj(&md, lin, (real)alpha, (real)kappa, Qr, Rr, yy, xb, Pb, &lp);
    if (rc) goto done;
    store(F, lp.F, T * n * n); store(c, lp.c, T * n); store(Qp, lp.Qp, T * n * n);
    store(H, lp.H, T * p * n); store(d, lp.d, T * p); store(Rp, lp.Rp, T * p * p); store(yt, lp.yt, T * p);
done:
    linpass_free(&lp);
    free(xb); free(Pb); free(yy);
    return rc;
}

/* One Kalman filter + RTS pass over a given surrogate model (arrays as returned
 * by orc_linearize_traj).  Outputs xf, Pf, xs, Ps over slots 0..T. */
int SFX(orc_kf_rts)(int nx, int ny, int T, const double *F, const double *c, const double *Qp,
                    const double *H, const double *d, const double *Rp, const double *yt,
                    const double *m0, const double *P0,
                    double *xf, double *Pf, double *xs, double *Ps) {
    if (nx < 1 || ny < 1 || nx > NMAX || ny > NMAX || T < 0) return ORC_EINVAL;
    int n = nx, p = ny;
    size_t S = (size_t)T + 1;
    linpass_t lp;
    real m0r[NMAX], P0r[NMAX * NMAX];
    real *a = malloc(sizeof(real) * S * n), *b = malloc(sizeof(real) * S * n * n);
    real *e = malloc(sizeof(real) * S * n), *f = malloc(sizeof(real) * S * n * n);
    int rc = linpass_alloc(&lp, n, p, T);
    if (rc || !a || !b || !e || !f) { rc = ORC_EINVAL; goto done; }
    load(lp.F, F, T * n * n); load(lp.c, c, T * n); load(lp.Qp, Qp, T * n * n);
    load(lp.H, H, T * p * n); load(lp.d, d, T * p); load(lp.Rp, Rp, T * p * p); load(lp.yt, yt, T * p);
    load(m0r, m0, n); load(P0r, P0, n * n);
    rc = kf_rts(&lp, m0r, P0r, 0, NULL, a, b, e, f);
    if (rc) goto done;
    store(xf, a, (int)(S * n)); store(Pf, b, (int)(S * n * n));
    store(xs, e, (int)(S * n)); store(Ps, f, (int)(S * n * n));
done:
    linpass_free(&lp);
    free(a); free(b); free(e); free(f);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Exported: the paper's parallel building blocks, one at a time.             */
/* Filtering element layout: [A (n*n), b (n), C (n*n), eta (n), J (n*n)].      */
/* Smoothing element layout: [E (n*n), g (n), L (n*n)].                        */
/* ------------------------------------------------------------------------ */

/*
 * Filtering element a_k (eq. 12-14) from the surrogate transition
 * (F_{k-1}, c_{k-1}, Q'_{k-1}) and measurement model (H_k, d_k, R'_k, y_k):
 *   S = H Q' H^T + R',  K = Q' H^T S^-1,
 *   A = (I - K H) F,  b = c + K (y - H c - d),  C = (I - K H) Q',
 *   J = (H F)^T S^-1 H F,  eta = (H F)^T S^-1 (y - H c - d).
 */
int SFX(orc_filter_element)(int nx, int ny, const double *F, const double *c, const double *Qp,
                            const double *H, const double *d, const double *Rp, const double *y,
                            double *out) {
    int n = nx, p = ny;
    if (n < 1 || p < 1 || n > NMAX || p > NMAX) return ORC_EINVAL;
    real Fr[NMAX * NMAX], cr[NMAX], Qr[NMAX * NMAX], Hr[NMAX * NMAX], dr[NMAX], Rr[NMAX * NMAX], yr[NMAX];
    load(Fr, F, n * n); load(cr, c, n); load(Qr, Qp, n * n); load(Hr, H, p * n); load(dr, d, p);
    load(Rr, Rp, p * p); load(yr, y, p);
    real QHt[NMAX * NMAX], S[NMAX * NMAX], L[NMAX * NMAX], Kt[NMAX * NMAX], IKH[NMAX * NMAX];
    real A[NMAX * NMAX], b[NMAX], C[NMAX * NMAX], HF[NMAX * NMAX], SiHF[NMAX * NMAX];
    real J[NMAX * NMAX], eta[NMAX], r[NMAX], Hc[NMAX], Sir[NMAX];
    mmt(n, n, p, Qr, Hr, QHt);
    mm(p, n, p, Hr, QHt, S);
    for (int i = 0; i < p * p; ++i) S[i] += Rr[i];
    symmetrize(p, S);
    if (chol(p, S, L)) return ORC_ENUMERIC;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < p; ++j) Kt[j * n + i] = QHt[i * p + j];
    chol_solve(p, L, Kt, n);                                  /* K^T */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            real s = (i == j);
            for (int t = 0; t < p; ++t) s -= Kt[t * n + i] * Hr[t * n + j];
            IKH[i * n + j] = s;
        }
    mm(n, n, n, IKH, Fr, A);
    mm(n, n, n, IKH, Qr, C);
    symmetrize(n, C);
    mv(p, n, Hr, cr, Hc);
    for (int j = 0; j < p; ++j) r[j] = yr[j] - Hc[j] - dr[j];
    for (int i = 0; i < n; ++i) {
        real s = cr[i];
        for (int j = 0; j < p; ++j) s += Kt[j * n + i] * r[j];
        b[i] = s;
    }
    mm(p, n, n, Hr, Fr, HF);
    memcpy(SiHF, HF, sizeof(real) * p * n);
    chol_solve(p, L, SiHF, n);
    mtm(n, p, n, HF, SiHF, J);
    symmetrize(n, J);
    memcpy(Sir, r, sizeof(real) * p);
    chol_solve(p, L, Sir, 1);
    for (int i = 0; i < n; ++i) {
        real s = 0;
        for (int j = 0; j < p; ++j) s += HF[j * n + i] * Sir[j];
        eta[i] = s;
    }
    store(out, A, n * n); store(out + n * n, b, n); store(out + n * n + n, C, n * n);
    store(out + 2 * n * n + n, eta, n); store(out + 2 * n * n + 2 * n, J, n * n);
    return ORC_OK;
}

/*
 * Filtering operator a_i (x) a_j (eq. 15):
 *   A_ij = A_j (I + C_i J_j)^-1 A_i
 *   b_ij = A_j (I + C_i J_j)^-1 (b_i + C_i eta_j) + b_j
 *   C_ij = A_j (I + C_i J_j)^-1 C_i A_j^T + C_j
 *   eta_ij = A_i^T (I + J_j C_i)^-1 (eta_j - J_j b_i) + eta_i
 *   J_ij = A_i^T (I + J_j C_i)^-1 J_j A_i + J_i
 */
int SFX(orc_filter_combine)(int n, const double *ai, const double *aj, double *out) {
    if (n < 1 || n > NMAX) return ORC_EINVAL;
    int nn = n * n;
    real Ai[NMAX * NMAX], bi[NMAX], Ci[NMAX * NMAX], ei[NMAX], Ji[NMAX * NMAX];
    real Aj[NMAX * NMAX], bj[NMAX], Cj[NMAX * NMAX], ej[NMAX], Jj[NMAX * NMAX];
    load(Ai, ai, nn); load(bi, ai + nn, n); load(Ci, ai + nn + n, nn); load(ei, ai + 2 * nn + n, n); load(Ji, ai + 2 * nn + 2 * n, nn);
    load(Aj, aj, nn); load(bj, aj + nn, n); load(Cj, aj + nn + n, nn); load(ej, aj + 2 * nn + n, n); load(Jj, aj + 2 * nn + 2 * n, nn);
    real D[NMAX * NMAX], rhs[NMAX * (2 * NMAX + 1)], CJ[NMAX * NMAX], Ce[NMAX];
    /* (I + C_i J_j) X = [A_i | b_i + C_i eta_j | C_i] */
    mm(n, n, n, Ci, Jj, CJ);
    for (int i = 0; i < nn; ++i) D[i] = CJ[i] + (i / n == i % n);
    mv(n, n, Ci, ej, Ce);
    int w = 2 * n + 1;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) rhs[i * w + j] = Ai[i * n + j];
        rhs[i * w + n] = bi[i] + Ce[i];
        for (int j = 0; j < n; ++j) rhs[i * w + n + 1 + j] = Ci[i * n + j];
    }
    if (gauss_solve(n, D, rhs, w)) return ORC_ENUMERIC;
    real X[NMAX * NMAX], xb[NMAX], XC[NMAX * NMAX], A[NMAX * NMAX], b[NMAX], C[NMAX * NMAX], t[NMAX * NMAX];
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) { X[i * n + j] = rhs[i * w + j]; XC[i * n + j] = rhs[i * w + n + 1 + j]; }
        xb[i] = rhs[i * w + n];
    }
    mm(n, n, n, Aj, X, A);
    mv(n, n, Aj, xb, b);
    for (int i = 0; i < n; ++i) b[i] += bj[i];
    mm(n, n, n, Aj, XC, t);
    mmt(n, n, n, t, Aj, C);
    for (int i = 0; i < nn; ++i) C[i] += Cj[i];
    symmetrize(n, C);
    /* (I + J_j C_i) Y = [eta_j - J_j b_i | J_j A_i] */
    real D2[NMAX * NMAX], rhs2[NMAX * (NMAX + 1)], JC[NMAX * NMAX], Jb[NMAX], JA[NMAX * NMAX];
    mm(n, n, n, Jj, Ci, JC);
    for (int i = 0; i < nn; ++i) D2[i] = JC[i] + (i / n == i % n);
    mv(n, n, Jj, bi, Jb);
    mm(n, n, n, Jj, Ai, JA);
    int w2 = n + 1;
    for (int i = 0; i < n; ++i) {
        rhs2[i * w2] = ej[i] - Jb[i];
        for (int j = 0; j < n; ++j) rhs2[i * w2 + 1 + j] = JA[i * n + j];
    }
    if (gauss_solve(n, D2, rhs2, w2)) return ORC_ENUMERIC;
    real ye[NMAX], YJ[NMAX * NMAX], eta[NMAX], J[NMAX * NMAX];
    for (int i = 0; i < n; ++i) {
        ye[i] = rhs2[i * w2];
        for (int j = 0; j < n; ++j) YJ[i * n + j] = rhs2[i * w2 + 1 + j];
    }
    for (int i = 0; i < n; ++i) {
        real s = ei[i];
        for (int t2 = 0; t2 < n; ++t2) s += Ai[t2 * n + i] * ye[t2];
        eta[i] = s;
    }
    mtm(n, n, n, Ai, YJ, J);
    for (int i = 0; i < nn; ++i) J[i] += Ji[i];
    symmetrize(n, J);
    store(out, A, nn); store(out + nn, b, n); store(out + nn + n, C, nn);
    store(out + 2 * nn + n, eta, n); store(out + 2 * nn + 2 * n, J, nn);
    return ORC_OK;
}

/*
 * Smoothing element (eq. 16-18) from the filtered (x*_k, P*_k) and the
 * surrogate transition (F_k, c_k, Q'_k) to slot k+1:
 *   E = P* F^T (F P* F^T + Q')^-1,  g = x* - E (F x* + c),  L = P* - E F P*.
 * last != 0 gives the end element E = 0, g = x*, L = P* (F, c, Qp unused).
 */
int SFX(orc_smoother_element)(int n, const double *xf, const double *Pf, const double *F,
                              const double *c, const double *Qp, int last, double *out) {
    if (n < 1 || n > NMAX) return ORC_EINVAL;
    int nn = n * n;
    real x[NMAX], P[NMAX * NMAX];
    load(x, xf, n); load(P, Pf, nn);
    real E[NMAX * NMAX] = {0}, g[NMAX], L[NMAX * NMAX];
    if (last) {
        memcpy(g, x, sizeof(real) * n);
        memcpy(L, P, sizeof(real) * nn);
    } else {
        real Fr[NMAX * NMAX], cr[NMAX], Qr[NMAX * NMAX], FP[NMAX * NMAX], Pp[NMAX * NMAX], Lc[NMAX * NMAX];
        real Et[NMAX * NMAX], Fx[NMAX], EFP[NMAX * NMAX];
        load(Fr, F, nn); load(cr, c, n); load(Qr, Qp, nn);
        mm(n, n, n, Fr, P, FP);
        mmt(n, n, n, FP, Fr, Pp);
        for (int i = 0; i < nn; ++i) Pp[i] += Qr[i];
        symmetrize(n, Pp);
        if (chol(n, Pp, Lc)) return ORC_ENUMERIC;
        memcpy(Et, FP, sizeof(real) * nn);          /* E^T = (F P F^T + Q')^-1 F P* */
        chol_solve(n, Lc, Et, n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) E[i * n + j] = Et[j * n + i];
        mv(n, n, Fr, x, Fx);
        for (int i = 0; i < n; ++i) Fx[i] += cr[i];
        for (int i = 0; i < n; ++i) {
            real s = x[i];
            for (int j = 0; j < n; ++j) s -= E[i * n + j] * Fx[j];
            g[i] = s;
        }
        mm(n, n, n, E, FP, EFP);
        for (int i = 0; i < nn; ++i) L[i] = P[i] - EFP[i];
        symmetrize(n, L);
    }
    store(out, E, nn); store(out + nn, g, n); store(out + nn + n, L, nn);
    return ORC_OK;
}

/* Smoothing operator a_i (x) a_j (eq. 19):
 *   E_ij = E_i E_j,  g_ij = E_i g_j + g_i,  L_ij = E_i L_j E_i^T + L_i. */
int SFX(orc_smoother_combine)(int n, const double *ai, const double *aj, double *out) {
    if (n < 1 || n > NMAX) return ORC_EINVAL;
    int nn = n * n;
    real Ei[NMAX * NMAX], gi[NMAX], Li[NMAX * NMAX], Ej[NMAX * NMAX], gj[NMAX], Lj[NMAX * NMAX];
    load(Ei, ai, nn); load(gi, ai + nn, n); load(Li, ai + nn + n, nn);
    load(Ej, aj, nn); load(gj, aj + nn, n); load(Lj, aj + nn + n, nn);
    real E[NMAX * NMAX], g[NMAX], t[NMAX * NMAX], L[NMAX * NMAX];
    mm(n, n, n, Ei, Ej, E);
    mv(n, n, Ei, gj, g);
    for (int i = 0; i < n; ++i) g[i] += gi[i];
    mm(n, n, n, Ei, Lj, t);
    mmt(n, n, n, t, Ei, L);
    for (int i = 0; i < nn; ++i) L[i] += Li[i];
    symmetrize(n, L);
    store(out, E, nn); store(out + nn, g, n); store(out + nn + n, L, nn);
    return ORC_OK;
}
