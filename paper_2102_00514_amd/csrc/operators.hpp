// The two associative operators of the method, per lane, on register tiles.
//
// Filtering (eq. 15), for a_i = (A_i, b_i, C_i, eta_i, J_i) followed by a_j:
//   A_ij = A_j (I + C_i J_j)^-1 A_i
//   b_ij = A_j (I + C_i J_j)^-1 (b_i + C_i eta_j) + b_j
//   C_ij = A_j (I + C_i J_j)^-1 C_i A_j^T + C_j
//   eta_ij = A_i^T (I + J_j C_i)^-1 (eta_j - J_j b_i) + eta_i
//   J_ij = A_i^T (I + J_j C_i)^-1 J_j A_i + J_i
// evaluated without forming or pivoting (I + C_i J_j): with C_i = U U^T
// (Cholesky) and G = I + U^T J_j U = Lg Lg^T (symmetric, eigenvalues >= 1),
//   M := (I + C_i J_j)^-1 C_i = U G^-1 U^T = W^T W,  W = Lg^-1 U^T,
//   (I + C_i J_j)^-1 = I - M J_j,   (I + J_j C_i)^-1 = I - J_j M.
// With Y = J_j A_i, Z = M Y, v = eta_j - J_j b_i and u = M v this gives
//   A_ij = A_j (A_i - Z),               J_ij = A_i^T Y - Y^T Z + J_i,
//   b_ij = A_j (b_i + u) + b_j,         eta_ij = A_i^T v - Y^T u + eta_i,
//   C_ij = A_j M A_j^T + C_j,
// where M, J_ij and C_ij are symmetric by construction (only the upper
// triangles are computed).
//
// Smoothing (eq. 19): (E_i, g_i, L_i) x (E_j, g_j, L_j) =
//   (E_i E_j, E_i g_j + g_i, E_i L_j E_i^T + L_i).
//
// Carries.  A filtering prefix that starts at a prior element (A = 0,
// eta = 0, J = 0) keeps A = eta = J = 0, so it is carried as (b, C) = the
// filtered mean and covariance; a smoothing suffix that ends at an end element
// (E = 0) is carried as (g, L) = the smoothed mean and covariance.
//
// Restarts.  A right operand whose A (filtering) or E (smoothing) is zero --
// a track's prior or end element, or any aggregate that contains one -- gives
// exactly (0, b_j, C_j) resp. (0, g_y, L_y) in those blocks, whatever the left
// operand holds.  The formulas give that only for finite operands (0 * NaN is
// NaN), so such an operand is taken as the result directly: a failed track
// never spills into the tracks that follow it in a batch.  eta and J of a
// restarted filtering result are the right operand's; they never reach b or C
// of any later result (those read b, C and A of a left operand, and a right
// operand with A = 0 restarts again).  Other results are unchanged.
//
// Scan order.  Both scans run left to right over "scan positions"; the
// smoothing scan visits slots from last to first, so its scan-order combine of
// an earlier position x with a later position y is y (x) x in the paper's order.
#pragma once

#include "linalg.hpp"

namespace pks {

template <int N, typename R>
struct FilterElem {
  R A[N][N], b[N], C[N][N], eta[N], J[N][N];
};
template <int N, typename R>
struct FilterCarry {
  R b[N], C[N][N];
};

// kIsolate = false drops the restart test, for scans over a single track
// (nothing follows a failed track there, and the test costs the ladders a few
// per cent).
template <int N, typename R, bool kIsolate = true>
struct FilterOp {
  // the scan ladders keep one copy of the operator instead of unrolling it
  static constexpr bool kCompact = false;
  using Elem = FilterElem<N, R>;
  using Carry = FilterCarry<N, R>;
  static constexpr int kS = sym_size<N>();
  static constexpr int kElemWords = N * N + 2 * N + 2 * kS;
  static constexpr int kCarryWords = N + kS;

  static PKS_DEV void load(const R* p, size_t st, size_t i, Elem& e) {
    ld_mat<N, N>(p, st, i, e.A);
    ld_vec<N>(p + N * N * st, st, i, e.b);
    ld_sym<N>(p + (N * N + N) * st, st, i, e.C);
    ld_vec<N>(p + (N * N + N + kS) * st, st, i, e.eta);
    ld_sym<N>(p + (N * N + 2 * N + kS) * st, st, i, e.J);
  }
  static PKS_DEV void store(R* p, size_t st, size_t i, const Elem& e) {
    st_mat<N, N>(p, st, i, e.A);
    st_vec<N>(p + N * N * st, st, i, e.b);
    st_sym<N>(p + (N * N + N) * st, st, i, e.C);
    st_vec<N>(p + (N * N + N + kS) * st, st, i, e.eta);
    st_sym<N>(p + (N * N + 2 * N + kS) * st, st, i, e.J);
  }
  static PKS_DEV void load(const R* p, size_t st, size_t i, Carry& c) {
    ld_vec<N>(p, st, i, c.b);
    ld_sym<N>(p + N * st, st, i, c.C);
  }
  static PKS_DEV void store(R* p, size_t st, size_t i, const Carry& c) {
    st_vec<N>(p, st, i, c.b);
    st_sym<N>(p + N * st, st, i, c.C);
  }
  // o = mv applied to every word of e: a lane move of the wavefront ladder,
  // in which every lane must take part.  The symmetric blocks move their
  // upper triangles only.
  template <class Mv>
  static PKS_DEV void move(const Elem& e, const Mv& mv, Elem& o) {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      o.b[i] = mv(e.b[i]);
      o.eta[i] = mv(e.eta[i]);
      PKS_UNROLL for (int j = 0; j < N; ++j) o.A[i][j] = mv(e.A[i][j]);
      PKS_UNROLL for (int j = i; j < N; ++j) {
        o.C[i][j] = o.C[j][i] = mv(e.C[i][j]);
        o.J[i][j] = o.J[j][i] = mv(e.J[i][j]);
      }
    }
  }

  // A carry-form element (prior element or a prefix from one): take (b, C).
  static PKS_DEV void to_carry(const Elem& e, Carry& c) {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      c.b[i] = e.b[i];
      PKS_UNROLL for (int j = 0; j < N; ++j) c.C[i][j] = e.C[i][j];
    }
  }

  static PKS_DEV bool restarts(const R (&A)[N][N]) {
    if constexpr (!kIsolate) {
      return false;
    } else {
      if (A[0][0] != R(0)) return false;
      bool z = true;
      PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) z &= A[i][j] == R(0);
      return z;
    }
  }

  // M = (I + C J)^-1 C, symmetric.  ok = false if C is not positive definite.
  static PKS_DEV bool core(const R (&Ci)[N][N], const R (&Jj)[N][N], R (&M)[N][N]) {
    R U[N][N], Ud[N];
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) U[i][j] = Ci[i][j];
    bool ok = chol_inplace<N>(U, Ud);
    // JU = J U (U lower triangular, true diagonal Ud)
    R JU[N][N];
    PKS_UNROLL for (int i = 0; i < N; ++i)
      PKS_UNROLL for (int k = 0; k < N; ++k) {
        R s = Jj[i][k] * Ud[k];
        PKS_UNROLL for (int t = k + 1; t < N; ++t) s += Jj[i][t] * U[t][k];
        JU[i][k] = s;
      }
    // G = I + U^T J U
    R G[N][N];
    PKS_UNROLL for (int a = 0; a < N; ++a)
      PKS_UNROLL for (int b = a; b < N; ++b) {
        R s = R(1) * (a == b) + Ud[a] * JU[a][b];
        PKS_UNROLL for (int t = a + 1; t < N; ++t) s += U[t][a] * JU[t][b];
        G[a][b] = s;
        G[b][a] = s;
      }
    ok = chol_inplace<N>(G) && ok;
    // W = Lg^-1 U^T (U^T upper triangular)
    R W[N][N];
    PKS_UNROLL for (int i = 0; i < N; ++i)
      PKS_UNROLL for (int j = 0; j < N; ++j) W[i][j] = (j > i) ? U[j][i] : (j == i ? Ud[i] : R(0));
    chol_fwd<N, N>(G, W);
    gram<N, N>(W, M);
    return ok;
  }

  // out = l (x) r
  static PKS_DEV void combine(const Elem& l, const Elem& r, Elem& o) {
    if (restarts(r.A)) {
      o = r;
      return;
    }
    R M[N][N];
    const bool ok = core(l.C, r.J, M);
    R Y[N][N], Z[N][N];
    mat_mul<N, N, N>(r.J, l.A, Y);
    mat_mul<N, N, N>(M, Y, Z);
    R v[N], u[N];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = r.eta[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) s -= r.J[i][t] * l.b[t];
      v[i] = s;
    }
    mat_vec<N, N>(M, v, u);
    // eta_ij = A_i^T v - Y^T u + eta_i
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = l.eta[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) s += l.A[t][i] * v[t] - Y[t][i] * u[t];
      o.eta[i] = s;
    }
    // J_ij = A_i^T Y - Y^T Z + J_i
    PKS_UNROLL for (int a = 0; a < N; ++a)
      PKS_UNROLL for (int b = a; b < N; ++b) {
        R s = l.J[a][b];
        PKS_UNROLL for (int t = 0; t < N; ++t) s += l.A[t][a] * Y[t][b] - Y[t][a] * Z[t][b];
        o.J[a][b] = s;
        o.J[b][a] = s;
      }
    // b_ij = A_j (b_i + u) + b_j
    PKS_UNROLL for (int i = 0; i < N; ++i) u[i] += l.b[i];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = r.b[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) s += r.A[i][t] * u[t];
      o.b[i] = s;
    }
    // A_ij = A_j (A_i - Z)
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Z[i][j] = l.A[i][j] - Z[i][j];
    mat_mul<N, N, N>(r.A, Z, o.A);
    // C_ij = A_j M A_j^T + C_j
    sandwich_add<N, N>(r.A, M, r.C, o.C);
    if (!ok) o.b[0] = quiet_nan<R>();
  }

  // out = c (x) r for a carry c
  static PKS_DEV void apply(const Carry& c, const Elem& r, Carry& o) {
    if (restarts(r.A)) {
      PKS_UNROLL for (int i = 0; i < N; ++i) {
        o.b[i] = r.b[i];
        PKS_UNROLL for (int j = 0; j < N; ++j) o.C[i][j] = r.C[i][j];
      }
      return;
    }
    R M[N][N];
    const bool ok = core(c.C, r.J, M);
    R v[N], u[N];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = r.eta[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) s -= r.J[i][t] * c.b[t];
      v[i] = s;
    }
    mat_vec<N, N>(M, v, u);
    PKS_UNROLL for (int i = 0; i < N; ++i) u[i] += c.b[i];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = r.b[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) s += r.A[i][t] * u[t];
      o.b[i] = s;
    }
    sandwich_add<N, N>(r.A, M, r.C, o.C);
    if (!ok) o.b[0] = quiet_nan<R>();
  }
};

template <int N, typename R>
struct SmootherElem {
  R E[N][N], g[N], L[N][N];
};
template <int N, typename R>
struct SmootherCarry {
  R g[N], L[N][N];
};

template <int N, typename R, bool kIsolate = true>
struct SmootherOp {
  // the scan ladders keep one copy of the operator instead of unrolling it
  static constexpr bool kCompact = false;
  using Elem = SmootherElem<N, R>;
  using Carry = SmootherCarry<N, R>;
  static constexpr int kS = sym_size<N>();
  static constexpr int kElemWords = N * N + N + kS;
  static constexpr int kCarryWords = N + kS;

  static PKS_DEV void load(const R* p, size_t st, size_t i, Elem& e) {
    ld_mat<N, N>(p, st, i, e.E);
    ld_vec<N>(p + N * N * st, st, i, e.g);
    ld_sym<N>(p + (N * N + N) * st, st, i, e.L);
  }
  static PKS_DEV void store(R* p, size_t st, size_t i, const Elem& e) {
    st_mat<N, N>(p, st, i, e.E);
    st_vec<N>(p + N * N * st, st, i, e.g);
    st_sym<N>(p + (N * N + N) * st, st, i, e.L);
  }
  static PKS_DEV void load(const R* p, size_t st, size_t i, Carry& c) {
    ld_vec<N>(p, st, i, c.g);
    ld_sym<N>(p + N * st, st, i, c.L);
  }
  static PKS_DEV void store(R* p, size_t st, size_t i, const Carry& c) {
    st_vec<N>(p, st, i, c.g);
    st_sym<N>(p + N * st, st, i, c.L);
  }
  template <class Mv>
  static PKS_DEV void move(const Elem& e, const Mv& mv, Elem& o) {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      o.g[i] = mv(e.g[i]);
      PKS_UNROLL for (int j = 0; j < N; ++j) o.E[i][j] = mv(e.E[i][j]);
      PKS_UNROLL for (int j = i; j < N; ++j) o.L[i][j] = o.L[j][i] = mv(e.L[i][j]);
    }
  }
  static PKS_DEV void to_carry(const Elem& e, Carry& c) {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      c.g[i] = e.g[i];
      PKS_UNROLL for (int j = 0; j < N; ++j) c.L[i][j] = e.L[i][j];
    }
  }
  static PKS_DEV bool restarts(const R (&E)[N][N]) {
    if constexpr (!kIsolate) {
      return false;
    } else {
      if (E[0][0] != R(0)) return false;
      bool z = true;
      PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) z &= E[i][j] == R(0);
      return z;
    }
  }
  // Scan order: x precedes y in the scan (x is the later slot); out = y (x) x.
  static PKS_DEV void combine(const Elem& x, const Elem& y, Elem& o) {
    if (restarts(y.E)) {
      PKS_UNROLL for (int i = 0; i < N; ++i) {
        o.g[i] = y.g[i];
        PKS_UNROLL for (int j = 0; j < N; ++j) {
          o.E[i][j] = R(0);
          o.L[i][j] = y.L[i][j];
        }
      }
      return;
    }
    mat_mul<N, N, N>(y.E, x.E, o.E);
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = y.g[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) s += y.E[i][t] * x.g[t];
      o.g[i] = s;
    }
    sandwich_add<N, N>(y.E, x.L, y.L, o.L);
  }
  static PKS_DEV void apply(const Carry& c, const Elem& y, Carry& o) {
    if (restarts(y.E)) {
      PKS_UNROLL for (int i = 0; i < N; ++i) {
        o.g[i] = y.g[i];
        PKS_UNROLL for (int j = 0; j < N; ++j) o.L[i][j] = y.L[i][j];
      }
      return;
    }
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = y.g[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) s += y.E[i][t] * c.g[t];
      o.g[i] = s;
    }
    sandwich_add<N, N>(y.E, c.L, y.L, o.L);
  }
};

}  // namespace pks
