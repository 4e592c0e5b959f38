// Device models of the additive-noise state-space model (eq. 4): the
// transition f and the measurement function h with their Jacobians.
//
//   LinearModel<N,P>      f(x) = F x + c, h(x) = H x + d       (test model)
//   CtBearings<N,P>       N/5 stacked coordinated-turn targets [px,py,vx,vy,w],
//                         P bearing sensors, sensor s sees target tgt(s)
//
// Parameters live in a device buffer whose pointer is uniform across the
// launch, so the compiler reads them through the scalar cache.
#pragma once

#include "linalg.hpp"

namespace pks {

template <typename R> PKS_DEV R two_pi() { return R(6.283185307179586476925286766559); }
template <typename R> PKS_DEV R pi_r() { return R(3.141592653589793238462643383279); }

PKS_DEV void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }
PKS_DEV void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }

// Angle difference folded into [-pi, pi).
template <typename R>
PKS_DEV R wrap_pi(R a) {
  return a - two_pi<R>() * floor((a + pi_r<R>()) / two_pi<R>());
}

template <int N_, int P_, typename R>
struct LinearModel {
  static constexpr int N = N_, P = P_;
  static constexpr bool kAngular = false;
  const R* prm;  // F (N*N), c (N), H (P*N), d (P)

  PKS_DEV void f(const R (&x)[N], R (&fx)[N]) const {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = prm[N * N + i];
      PKS_UNROLL for (int j = 0; j < N; ++j) s += prm[i * N + j] * x[j];
      fx[i] = s;
    }
  }
  PKS_DEV void f_jac(const R (&x)[N], R (&fx)[N], R (&Fx)[N][N]) const {
    f(x, fx);
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Fx[i][j] = prm[i * N + j];
  }
  PKS_DEV void h(const R (&x)[N], R (&hx)[P]) const {
    const R* H = prm + N * N + N;
    PKS_UNROLL for (int i = 0; i < P; ++i) {
      R s = H[P * N + i];
      PKS_UNROLL for (int j = 0; j < N; ++j) s += H[i * N + j] * x[j];
      hx[i] = s;
    }
  }
  PKS_DEV void h_jac(const R (&x)[N], R (&hx)[P], R (&Hx)[P][N]) const {
    h(x, hx);
    const R* H = prm + N * N + N;
    PKS_UNROLL for (int i = 0; i < P; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Hx[i][j] = H[i * N + j];
  }
};

// Coefficients of the coordinated-turn transition for a = w*dt:
//   s1 = sin(a)/w, s2 = (1 - cos a)/w, their w-derivatives d1, d2, and sin a, cos a.
// Small |a| uses truncated power series (exact limit at w = 0, truncation
// below 1e-18 relative for |a| < 0.1); otherwise the closed forms, with
// 1 - cos a evaluated as 2 sin^2(a/2).
template <typename R>
PKS_DEV void ct_terms(R w, R dt, R& s1, R& s2, R& d1, R& d2, R& sa, R& ca) {
  const R a = w * dt;
  const R a2 = a * a;
  if (fabs(a) < R(0.1)) {
    // sin(a)/a and (1-cos a)/a^2 as polynomials in a^2
    const R sinc = R(1) + a2 * (R(-1) / 6 + a2 * (R(1) / 120 + a2 * (R(-1) / 5040 + a2 * (R(1) / 362880))));
    const R cosc = R(0.5) + a2 * (R(-1) / 24 + a2 * (R(1) / 720 + a2 * (R(-1) / 40320 + a2 * (R(1) / 3628800))));
    s1 = dt * sinc;
    s2 = dt * a * cosc;
    sa = a * sinc;
    ca = R(1) - a2 * cosc;
    // d/da of sinc and of a*cosc
    d1 = dt * dt * a * (R(-1) / 3 + a2 * (R(1) / 30 + a2 * (R(-1) / 840 + a2 * (R(1) / 45360 + a2 * (R(-1) / 3991680)))));
    d2 = dt * dt * (R(0.5) + a2 * (R(-1) / 8 + a2 * (R(1) / 144 + a2 * (R(-1) / 5760 + a2 * (R(1) / 403200)))));
  } else {
    R sh, chh;
    sin_cos(a * R(0.5), &sh, &chh);
    sa = R(2) * sh * chh;
    const R omc = R(2) * sh * sh;
    ca = R(1) - omc;
    const R inv_w = rcp_nr(w);
    s1 = sa * inv_w;
    s2 = omc * inv_w;
    const R k = dt * dt * rcp_nr(a2);
    d1 = k * (a * ca - sa);
    d2 = k * (a * sa - omc);
  }
}

template <int N_, int P_, typename R>
struct CtBearings {
  static constexpr int N = N_, P = P_;
  static constexpr int NT = N / 5;
  static_assert(N % 5 == 0, "coordinated-turn state is made of 5-blocks");
  static constexpr bool kAngular = true;
  const R* prm;  // dt, (sx, sy, target) * P

  PKS_DEV R dt() const { return prm[0]; }

  template <bool kJac>
  PKS_DEV void f_impl(const R (&x)[N], R (&fx)[N], R (*Fx)[N]) const {
    const R h = dt();
    PKS_UNROLL for (int b = 0; b < NT; ++b) {
      const int o = 5 * b;
      const R vx = x[o + 2], vy = x[o + 3], w = x[o + 4];
      R s1, s2, d1, d2, sa, ca;
      ct_terms<R>(w, h, s1, s2, d1, d2, sa, ca);
      fx[o + 0] = x[o + 0] + s1 * vx - s2 * vy;
      fx[o + 1] = x[o + 1] + s2 * vx + s1 * vy;
      fx[o + 2] = ca * vx - sa * vy;
      fx[o + 3] = sa * vx + ca * vy;
      fx[o + 4] = w;
      if constexpr (kJac) {
        PKS_UNROLL for (int i = 0; i < 5; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Fx[o + i][j] = R(0);
        Fx[o + 0][o + 0] = R(1);
        Fx[o + 0][o + 2] = s1;
        Fx[o + 0][o + 3] = -s2;
        Fx[o + 0][o + 4] = d1 * vx - d2 * vy;
        Fx[o + 1][o + 1] = R(1);
        Fx[o + 1][o + 2] = s2;
        Fx[o + 1][o + 3] = s1;
        Fx[o + 1][o + 4] = d2 * vx + d1 * vy;
        Fx[o + 2][o + 2] = ca;
        Fx[o + 2][o + 3] = -sa;
        Fx[o + 2][o + 4] = -h * fx[o + 3];
        Fx[o + 3][o + 2] = sa;
        Fx[o + 3][o + 3] = ca;
        Fx[o + 3][o + 4] = h * fx[o + 2];
        Fx[o + 4][o + 4] = R(1);
      }
    }
  }
  PKS_DEV void f(const R (&x)[N], R (&fx)[N]) const { f_impl<false>(x, fx, nullptr); }
  PKS_DEV void f_jac(const R (&x)[N], R (&fx)[N], R (&Fx)[N][N]) const { f_impl<true>(x, fx, Fx); }

  // Position of the target seen by sensor s, selected without dynamic indexing.
  PKS_DEV void target_pos(const R (&x)[N], int t, R& px, R& py) const {
    px = x[0];
    py = x[1];
    PKS_UNROLL for (int b = 1; b < NT; ++b) {
      px = (t == b) ? x[5 * b] : px;
      py = (t == b) ? x[5 * b + 1] : py;
    }
  }

  PKS_DEV void h(const R (&x)[N], R (&hx)[P]) const {
    PKS_UNROLL for (int s = 0; s < P; ++s) {
      const R sx = prm[1 + 3 * s], sy = prm[2 + 3 * s];
      const int t = int(prm[3 + 3 * s]);
      R px, py;
      target_pos(x, t, px, py);
      hx[s] = atan2(py - sy, px - sx);
    }
  }
  PKS_DEV void h_jac(const R (&x)[N], R (&hx)[P], R (&Hx)[P][N]) const {
    PKS_UNROLL for (int s = 0; s < P; ++s) {
      const R sx = prm[1 + 3 * s], sy = prm[2 + 3 * s];
      const int t = int(prm[3 + 3 * s]);
      R px, py;
      target_pos(x, t, px, py);
      const R dx = px - sx, dy = py - sy;
      hx[s] = atan2(dy, dx);
      const R ir2 = rcp_nr(dx * dx + dy * dy);
      PKS_UNROLL for (int j = 0; j < N; ++j) Hx[s][j] = R(0);
      PKS_UNROLL for (int b = 0; b < NT; ++b) {
        Hx[s][5 * b] = (t == b) ? -dy * ir2 : R(0);
        Hx[s][5 * b + 1] = (t == b) ? dx * ir2 : R(0);
      }
    }
  }
};

}  // namespace pks
