// Per-slot work of one iteration: linearisation around the previous smoothed
// trajectory (Section 3), the filtering element (eq. 12-14) and the smoothing
// element (eq. 16-18).  Everything is evaluated by one lane for one slot.
#pragma once

#include "linalg.hpp"
#include "models.hpp"

namespace pks {

enum LinKind : int { kTaylor = 0, kCubature = 1, kUnscented = 2 };

struct SigmaRule {
  double alpha, kappa;  // unscented lambda = alpha^2 (n + kappa) - n
};

template <int N, typename R>
PKS_DEV void sigma_weights(int lin, SigmaRule rule, R& spread, R& w0, R& wj) {
  if (lin == kCubature) {
    spread = sqrt(R(N));
    w0 = R(0);
    wj = R(1) / R(2 * N);
  } else {
    const R lam = R(rule.alpha * rule.alpha * (N + rule.kappa) - N);
    spread = sqrt(R(N) + lam);
    w0 = lam / (R(N) + lam);
    wj = R(1) / (R(2) * (R(N) + lam));
  }
}

// ---------------------------------------------------------------------------
// Statistical linear regression of g: R^N -> R^Q at N(xbar, Pbar) (eq. 7-9).
//
// With the symmetric point set X_j^(+/-) = xbar +/- gamma L e_j (L = chol Pbar,
// lower) plus an optional centre point, the cross moment is
//     Psi = sum_j w_j gamma L e_j (Z_j^+ - Z_j^-)^T = L Delta,
// so G = Psi^T Pbar^-1 = Delta^T L^-1 and G Pbar G^T = Delta^T Delta.  The
// regression therefore needs one triangular solve and no inverse of Pbar.
// Eval(x, z) writes g(x); for angular outputs each image is unwrapped around
// zc = g(xbar).
// ---------------------------------------------------------------------------
template <int N, int Q, bool kAngular, typename R, class Eval>
PKS_DEV bool slr(int lin, SigmaRule rule, const R (&xbar)[N], const R (&Pbar)[N][N], Eval eval,
                 R (&G)[Q][N], R (&g)[Q], R (&Lam)[Q][Q], R (&zc)[Q]) {
  R L[N][N];
  PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) L[i][j] = Pbar[i][j];
  R Ld[N];  // diagonal of the factor (L itself keeps the reciprocals)
  const bool ok = chol_inplace<N>(L, Ld);
  R gamma, w0, wj;
  sigma_weights<N, R>(lin, rule, gamma, w0, wj);
  eval(xbar, zc);
  R Zp[N][Q], Zm[N][Q];
  PKS_UNROLL for (int j = 0; j < N; ++j) {
    R xp[N], xm[N];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      const R lij = (i == j) ? Ld[j] : (i > j ? L[i][j] : R(0));
      xp[i] = xbar[i] + gamma * lij;
      xm[i] = xbar[i] - gamma * lij;
    }
    R zp[Q], zm[Q];
    eval(xp, zp);
    eval(xm, zm);
    PKS_UNROLL for (int q = 0; q < Q; ++q) {
      if constexpr (kAngular) {
        zp[q] = zc[q] + wrap_pi<R>(zp[q] - zc[q]);
        zm[q] = zc[q] + wrap_pi<R>(zm[q] - zc[q]);
      }
      Zp[j][q] = zp[q];
      Zm[j][q] = zm[q];
    }
  }
  // mean of the images
  PKS_UNROLL for (int q = 0; q < Q; ++q) {
    R s = R(0);
    PKS_UNROLL for (int j = 0; j < N; ++j) s += Zp[j][q] + Zm[j][q];
    g[q] = w0 * zc[q] + wj * s;
  }
  // Delta_j = w_j gamma (Z_j^+ - Z_j^-)
  R D[N][Q];
  const R wg = wj * gamma;
  PKS_UNROLL for (int j = 0; j < N; ++j) PKS_UNROLL for (int q = 0; q < Q; ++q) D[j][q] = wg * (Zp[j][q] - Zm[j][q]);
  // Lambda = Phi - G Pbar G^T = Phi - Delta^T Delta, evaluated as the weighted
  // sum of outer products of the regression residuals
  //   r_j^(+/-) = (Z_j^(+/-) - zbar) - G (X_j^(+/-) - xbar) = Z_j^(+/-) - zbar -/+ gamma Delta_j,
  //   r_0 = zc - zbar (centre point).
  // The two forms are equal; this one is positive semi-definite by
  // construction (non-negative weights), where the difference of two nearly
  // equal matrices can lose definiteness in FP32.
  PKS_UNROLL for (int j = 0; j < N; ++j)
    PKS_UNROLL for (int q = 0; q < Q; ++q) {
      Zp[j][q] = Zp[j][q] - g[q] - gamma * D[j][q];
      Zm[j][q] = Zm[j][q] - g[q] + gamma * D[j][q];
    }
  PKS_UNROLL for (int a = 0; a < Q; ++a)
    PKS_UNROLL for (int b = a; b < Q; ++b) {
      R s = R(0);
      PKS_UNROLL for (int j = 0; j < N; ++j) s += Zp[j][a] * Zp[j][b] + Zm[j][a] * Zm[j][b];
      s *= wj;
      s += w0 * (zc[a] - g[a]) * (zc[b] - g[b]);
      Lam[a][b] = s;
      Lam[b][a] = s;
    }
  // G^T = L^-T Delta
  chol_bwd<N, Q>(L, D);
  PKS_UNROLL for (int q = 0; q < Q; ++q) PKS_UNROLL for (int i = 0; i < N; ++i) G[q][i] = D[i][q];
  // offset: g = zbar - G xbar
  PKS_UNROLL for (int q = 0; q < Q; ++q) {
    R s = g[q];
    PKS_UNROLL for (int i = 0; i < N; ++i) s -= G[q][i] * xbar[i];
    g[q] = s;
  }
  return ok;
}

// Transition linearisation at slot k: F_k, c_k and Q'_k = Q + Lambda_k (eq. 10 / eq. 7, 11).
template <class Model, typename R>
PKS_DEV bool linearize_f(const Model& md, int lin, SigmaRule rule, const R (&Q)[Model::N][Model::N],
                         const R (&xbar)[Model::N], const R (&Pbar)[Model::N][Model::N],
                         R (&F)[Model::N][Model::N], R (&c)[Model::N], R (&Qp)[Model::N][Model::N]) {
  constexpr int N = Model::N;
  if (lin == kTaylor) {
    R fx[N];
    md.f_jac(xbar, fx, F);
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = fx[i];
      PKS_UNROLL for (int j = 0; j < N; ++j) s -= F[i][j] * xbar[j];
      c[i] = s;
    }
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Qp[i][j] = Q[i][j];
    return true;
  }
  R Lam[N][N], zc[N];
  const bool ok = slr<N, N, false, R>(lin, rule, xbar, Pbar,
                                      [&](const R (&x)[N], R (&z)[N]) { md.f(x, z); }, F, c, Lam, zc);
  PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Qp[i][j] = Q[i][j] + Lam[i][j];
  return ok;
}

// Measurement linearisation at slot k: H_k, d_k, R'_k = R + Omega_k and the
// measurement ytil_k, unwrapped around h(xbar_k) for angular models.
template <class Model, typename R>
PKS_DEV bool linearize_h(const Model& md, int lin, SigmaRule rule, const R (&Rm)[Model::P][Model::P],
                         const R (&xbar)[Model::N], const R (&Pbar)[Model::N][Model::N], const R (&y)[Model::P],
                         R (&H)[Model::P][Model::N], R (&d)[Model::P], R (&Rp)[Model::P][Model::P],
                         R (&yt)[Model::P]) {
  constexpr int N = Model::N, P = Model::P;
  R hc[P];
  bool ok = true;
  if (lin == kTaylor) {
    md.h_jac(xbar, hc, H);
    PKS_UNROLL for (int i = 0; i < P; ++i) {
      R s = hc[i];
      PKS_UNROLL for (int j = 0; j < N; ++j) s -= H[i][j] * xbar[j];
      d[i] = s;
    }
    PKS_UNROLL for (int i = 0; i < P; ++i) PKS_UNROLL for (int j = 0; j < P; ++j) Rp[i][j] = Rm[i][j];
  } else {
    R Om[P][P];
    ok = slr<N, P, Model::kAngular, R>(lin, rule, xbar, Pbar,
                                       [&](const R (&x)[N], R (&z)[P]) { md.h(x, z); }, H, d, Om, hc);
    PKS_UNROLL for (int i = 0; i < P; ++i) PKS_UNROLL for (int j = 0; j < P; ++j) Rp[i][j] = Rm[i][j] + Om[i][j];
  }
  PKS_UNROLL for (int i = 0; i < P; ++i) yt[i] = Model::kAngular ? hc[i] + wrap_pi<R>(y[i] - hc[i]) : y[i];
  return ok;
}

// ---------------------------------------------------------------------------
// Filtering element a_k = (A, b, C, eta, J) (eq. 13-14) from the surrogate
// transition (F, c, Q') into slot k and measurement (H, d, R', y) at slot k.
// With S = H Q' H^T + R' = L L^T, Z = L^-1 H Q', Y = L^-1 H F, w = L^-1 (y - H c - d):
//   K = Q' H^T S^-1 = Z^T L^-1, so
//   A = F - Z^T Y,  b = c + Z^T w,  C = Q' - Z^T Z,  J = Y^T Y,  eta = Y^T w.
// ---------------------------------------------------------------------------
template <int N, int P, typename R>
PKS_DEV bool filter_element(const R (&F)[N][N], const R (&c)[N], const R (&Qp)[N][N],
                            const R (&H)[P][N], const R (&d)[P], const R (&Rp)[P][P], const R (&y)[P],
                            R (&A)[N][N], R (&b)[N], R (&C)[N][N], R (&eta)[N], R (&J)[N][N]) {
  R HQ[P][N], HF[P][N], S[P][P];
  mat_mul<P, N, N>(H, Qp, HQ);
  mat_mul<P, N, N>(H, F, HF);
  PKS_UNROLL for (int i = 0; i < P; ++i)
    PKS_UNROLL for (int j = i; j < P; ++j) {
      R s = Rp[i][j];
      PKS_UNROLL for (int t = 0; t < N; ++t) s += HQ[i][t] * H[j][t];
      S[i][j] = s;
      S[j][i] = s;
    }
  const bool ok = chol_inplace<P>(S);
  R w[P];
  PKS_UNROLL for (int i = 0; i < P; ++i) {
    R s = y[i] - d[i];
    PKS_UNROLL for (int t = 0; t < N; ++t) s -= H[i][t] * c[t];
    w[i] = s;
  }
  chol_fwd<P, N>(S, HQ);  // Z
  chol_fwd<P, N>(S, HF);  // Y
  chol_fwd_vec<P>(S, w);
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R sb = c[i], se = R(0);
    PKS_UNROLL for (int t = 0; t < P; ++t) {
      sb += HQ[t][i] * w[t];
      se += HF[t][i] * w[t];
    }
    b[i] = sb;
    eta[i] = se;
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      R sa = F[i][j];
      PKS_UNROLL for (int t = 0; t < P; ++t) sa -= HQ[t][i] * HF[t][j];
      A[i][j] = sa;
    }
    PKS_UNROLL for (int j = i; j < N; ++j) {
      R sc = Qp[i][j], sj = R(0);
      PKS_UNROLL for (int t = 0; t < P; ++t) {
        sc -= HQ[t][i] * HQ[t][j];
        sj += HF[t][i] * HF[t][j];
      }
      C[i][j] = sc;
      C[j][i] = sc;
      J[i][j] = sj;
      J[j][i] = sj;
    }
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Levenberg-Marquardt damping (Section 3, the damped Gauss-Newton extension of
// the iterated smoother): the previous iterate xbar_k is observed at slot k
// through x_k plus noise of covariance I/lambda.  That measurement is
// independent of y_k given x_k, so it is a second update of the filtering
// element.  With G = I + lambda C = L L^T, Z = L^-1 C, W = L^-1 A and
// v = L^-1 (xbar - b), the gain is K = C (C + I/lambda)^-1 = lambda Z^T L^-1 and
//   A -= lambda Z^T W,  b += lambda Z^T v,  C -= lambda Z^T Z,
//   J += lambda W^T W,  eta += lambda W^T v.
// Returns false if G is not positive definite.
// ---------------------------------------------------------------------------
template <int N, typename R>
PKS_DEV bool lm_damp_element(R lam, const R (&xbar)[N], R (&A)[N][N], R (&b)[N], R (&C)[N][N], R (&eta)[N],
                             R (&J)[N][N]) {
  R G[N][N], Z[N][N], W[N][N], v[N];
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    v[i] = xbar[i] - b[i];
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      G[i][j] = lam * C[i][j] + (i == j ? R(1) : R(0));
      Z[i][j] = C[i][j];
      W[i][j] = A[i][j];
    }
  }
  const bool ok = chol_inplace<N>(G);
  chol_fwd<N, N>(G, Z);
  chol_fwd<N, N>(G, W);
  chol_fwd_vec<N>(G, v);
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R sb = R(0), se = R(0);
    PKS_UNROLL for (int t = 0; t < N; ++t) {
      sb += Z[t][i] * v[t];
      se += W[t][i] * v[t];
    }
    b[i] += lam * sb;
    eta[i] += lam * se;
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      R sa = R(0);
      PKS_UNROLL for (int t = 0; t < N; ++t) sa += Z[t][i] * W[t][j];
      A[i][j] -= lam * sa;
    }
    PKS_UNROLL for (int j = i; j < N; ++j) {
      R sc = R(0), sj = R(0);
      PKS_UNROLL for (int t = 0; t < N; ++t) {
        sc += Z[t][i] * Z[t][j];
        sj += W[t][i] * W[t][j];
      }
      C[i][j] -= lam * sc;
      C[j][i] = C[i][j];
      J[i][j] += lam * sj;
      J[j][i] = J[i][j];
    }
  }
  return ok;
}

// The same damping update applied to filtered moments (m, P) of the
// sequential Kalman filter: m += lambda Z^T v, P -= lambda Z^T Z with
// G = I + lambda P = L L^T, Z = L^-1 P, v = L^-1 (xbar - m).
template <int N, typename R>
PKS_DEV bool lm_damp_moments(R lam, const R (&xbar)[N], R (&m)[N], R (&P)[N][N]) {
  R G[N][N], Z[N][N], v[N];
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    v[i] = xbar[i] - m[i];
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      G[i][j] = lam * P[i][j] + (i == j ? R(1) : R(0));
      Z[i][j] = P[i][j];
    }
  }
  const bool ok = chol_inplace<N>(G);
  chol_fwd<N, N>(G, Z);
  chol_fwd_vec<N>(G, v);
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R sb = R(0);
    PKS_UNROLL for (int t = 0; t < N; ++t) sb += Z[t][i] * v[t];
    m[i] += lam * sb;
    PKS_UNROLL for (int j = i; j < N; ++j) {
      R sc = R(0);
      PKS_UNROLL for (int t = 0; t < N; ++t) sc += Z[t][i] * Z[t][j];
      P[i][j] -= lam * sc;
      P[j][i] = P[i][j];
    }
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Smoothing element (E, g, L) (eq. 17) from the filtered x*, P* at slot k and
// the surrogate transition (F, c, Q') out of slot k.  With
// F P* F^T + Q' = L L^T and V = L^-1 F P*:
//   E = P* F^T (F P* F^T + Q')^-1 = V^T L^-1,  g = x* - E (F x* + c),
//   L_k = P* - E F P* = P* - V^T V.
// ---------------------------------------------------------------------------
template <int N, typename R>
PKS_DEV bool smoother_element(const R (&xf)[N], const R (&Pf)[N][N], const R (&F)[N][N], const R (&c)[N],
                              const R (&Qp)[N][N], R (&E)[N][N], R (&g)[N], R (&Ls)[N][N]) {
  R FP[N][N], Pp[N][N];
  mat_mul<N, N, N>(F, Pf, FP);
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = i; j < N; ++j) {
      R s = Qp[i][j];
      PKS_UNROLL for (int t = 0; t < N; ++t) s += FP[i][t] * F[j][t];
      Pp[i][j] = s;
      Pp[j][i] = s;
    }
  const bool ok = chol_inplace<N>(Pp);
  R r[N];
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R s = c[i];
    PKS_UNROLL for (int t = 0; t < N; ++t) s += F[i][t] * xf[t];
    r[i] = s;
  }
  chol_fwd<N, N>(Pp, FP);  // V
  chol_fwd_vec<N>(Pp, r);  // L^-1 (F x* + c)
  // L_k = P* - V^T V
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = i; j < N; ++j) {
      R s = Pf[i][j];
      PKS_UNROLL for (int t = 0; t < N; ++t) s -= FP[t][i] * FP[t][j];
      Ls[i][j] = s;
      Ls[j][i] = s;
    }
  // g = x* - V^T L^-1 (F x* + c)
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R s = xf[i];
    PKS_UNROLL for (int t = 0; t < N; ++t) s -= FP[t][i] * r[t];
    g[i] = s;
  }
  // E^T = L^-T V
  chol_bwd<N, N>(Pp, FP);
  PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) E[i][j] = FP[j][i];
  return ok;
}

}  // namespace pks
