// Square-root (Cholesky-factor) form of the filtering and smoothing elements
// and of their associative operators.
//
// Every covariance-like block is carried as a lower-triangular factor:
// C = U U^T and J = Z Z^T in the filtering elements, L = D D^T in the
// smoothing elements.  New factors come from tria(X): the lower-triangular
// factor of X X^T obtained from an LQ decomposition of X (Householder
// reflections from the right), so no covariance is ever formed and then
// factorised, no difference of two covariances is taken, and no step can
// fail for lack of definiteness.  The operators are algebraically those of
// eq. 15 and eq. 19; the elements those of eq. 13-14 and eq. 16-18.
//
// Filtering operator.  For a_i (x) a_j put B = U_i^T Z_j and
//   Xi = tria([B, I]),  Phi = tria([B^T, I])        (Xi Xi^T = I + U_i^T J_j U_i)
//   W = U_i Xi^-T,  V = Xi^-1 B Z_j^T,  Xi22 = Z_j Phi^-T.
// Then (I + C_i J_j)^-1 = I - W V, (I + C_i J_j)^-1 C_i = W W^T and
// (I + J_j C_i)^-1 J_j = Xi22 Xi22^T (push-through identity), so
//   A_ij = A_j (A_i - W (V A_i))
//   b_ij = A_j (b_i + W (W^T eta_j - V b_i)) + b_j
//   U_ij = tria([A_j W, U_j])
//   eta_ij = A_i^T (s - V^T (W^T s)) + eta_i, s = eta_j - Z_j (Z_j^T b_i)
//   Z_ij = tria([A_i^T Xi22, Z_i]).
// Xi and Phi have eigenvalues >= 1, so the triangular solves are benign.
//
// Smoothing operator: (E_i, g_i, D_i) x (E_j, g_j, D_j) =
//   (E_i E_j, E_i g_j + g_i, tria([E_i D_j, D_i])).
//
// Carries, restarts and scan order are as for the covariance form
// (operators.hpp): prior elements have A = 0, end elements E = 0.
#pragma once

#include "linalg.hpp"
#include "operators.hpp"

namespace pks {

// ---------------------------------------------------------------------------
// tria: lower-triangular L (M x M, non-negative diagonal) with L L^T = X X^T
// for X of M x K, K >= M.  Row r of X is reduced by one Householder
// reflection acting on columns r..K-1, applied to every later row.  X is
// destroyed.  A zero row remainder (rank deficiency) gives a zero column.
// ---------------------------------------------------------------------------
template <int M, int K, typename R>
PKS_DEV void tria(R (&X)[M][K], R (&L)[M][M]) {
  static_assert(K >= M, "tria needs at least as many columns as rows");
  PKS_UNROLL for (int r = 0; r < M; ++r) {
    R ss = R(0);
    PKS_UNROLL for (int j = r; j < K; ++j) ss += X[r][j] * X[r][j];
    const bool nz = ss > R(0);
    const R inv = rsqrt_nr(nz ? ss : R(1));
    const R nrm = nz ? ss * inv : R(0);                 // |x|
    const R x0 = X[r][r];
    const R sg = x0 < R(0) ? R(-1) : R(1);
    // v = x + sign(x0) |x| e_0;  H = I - beta v v^T with beta = 1 / (|x| (|x| + |x0|))
    const R v0 = x0 + sg * nrm;
    const R den = nrm * (nrm + sg * x0);
    const R beta = nz ? rcp_nr(den > R(0) ? den : R(1)) : R(0);
    PKS_UNROLL for (int i = r + 1; i < M; ++i) {
      R dot = X[i][r] * v0;
      PKS_UNROLL for (int j = r + 1; j < K; ++j) dot += X[i][j] * X[r][j];
      const R f = beta * dot;
      X[i][r] -= f * v0;
      PKS_UNROLL for (int j = r + 1; j < K; ++j) X[i][j] -= f * X[r][j];
    }
    // the reflected row is (-sign(x0) |x|, 0, ..., 0); flipping the sign of
    // column r (of L) leaves L L^T unchanged and makes the diagonal |x|
    L[r][r] = nrm;
    PKS_UNROLL for (int i = r + 1; i < M; ++i) L[i][r] = -sg * X[i][r];
    PKS_UNROLL for (int j = r + 1; j < M; ++j) L[r][j] = R(0);
  }
}

// X (M x K) = [A, B] for A (M x K1), B (M x K2), K = K1 + K2.
template <int M, int K1, int K2, typename R>
PKS_DEV void hcat(const R (&A)[M][K1], const R (&B)[M][K2], R (&X)[M][K1 + K2]) {
  PKS_UNROLL for (int i = 0; i < M; ++i) {
    PKS_UNROLL for (int j = 0; j < K1; ++j) X[i][j] = A[i][j];
    PKS_UNROLL for (int j = 0; j < K2; ++j) X[i][K1 + j] = B[i][j];
  }
}

// Solve L Y = B (L lower triangular with its true diagonal), M right-hand
// sides stored as columns of B (N x M), in place.
template <int N, int M, typename R>
PKS_DEV void tril_solve(const R (&L)[N][N], R (&B)[N][M]) {
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    const R inv = rcp_nr(L[i][i]);
    PKS_UNROLL for (int c = 0; c < M; ++c) {
      R s = B[i][c];
      PKS_UNROLL for (int t = 0; t < i; ++t) s -= L[i][t] * B[t][c];
      B[i][c] = s * inv;
    }
  }
}

// Solve L^T Y = B (L lower triangular with its true diagonal), in place.
template <int N, int M, typename R>
PKS_DEV void tril_tsolve(const R (&L)[N][N], R (&B)[N][M]) {
  PKS_UNROLL for (int i = N - 1; i >= 0; --i) {
    const R inv = rcp_nr(L[i][i]);
    PKS_UNROLL for (int c = 0; c < M; ++c) {
      R s = B[i][c];
      PKS_UNROLL for (int t = i + 1; t < N; ++t) s -= L[t][i] * B[t][c];
      B[i][c] = s * inv;
    }
  }
}

// Lower-triangular factor with its true diagonal: A = L L^T.  Returns false
// if a pivot is not positive.
template <int N, typename R>
PKS_DEV bool chol_lower(const R (&A)[N][N], R (&L)[N][N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) L[i][j] = A[i][j];
  R d[N];
  const bool ok = chol_inplace<N>(L, d);
  PKS_UNROLL for (int j = 0; j < N; ++j) {
    L[j][j] = d[j];
    PKS_UNROLL for (int i = 0; i < j; ++i) L[i][j] = R(0);
  }
  return ok;
}

// Lower-triangular factor L L^T = A of a symmetric positive semi-definite A
// (a transition covariance Q' with a noise-free state component).  A pivot at
// or below 64 eps times the largest diagonal entry is a direction without
// variance: its column is set to zero, which tria and the operators on
// factors accept (eq. 15 needs I + C_i J_j invertible, not C_i definite).
// For a well-conditioned positive definite A no pivot is that small and the
// result is chol_lower's.  Returns false if a pivot is below minus that bound
// or not finite.
template <int N, typename R>
PKS_DEV bool chol_lower_psd(const R (&A)[N][N], R (&L)[N][N]) {
  constexpr R kEps = sizeof(R) == 8 ? R(2.220446049250313e-16) : R(1.1920929e-7);
  R dmax = R(0);
  PKS_UNROLL for (int i = 0; i < N; ++i) dmax = A[i][i] > dmax ? A[i][i] : dmax;
  const R tiny = R(64) * kEps * dmax;
  bool ok = true;
  PKS_UNROLL for (int j = 0; j < N; ++j) {
    R s = A[j][j];
    PKS_UNROLL for (int t = 0; t < j; ++t) s -= L[j][t] * L[j][t];
    ok = ok && (s >= -tiny);   // false for NaN
    const R inv = s > tiny ? rsqrt_nr(s) : R(0);
    L[j][j] = s * inv;
    PKS_UNROLL for (int i = j + 1; i < N; ++i) {
      R v = A[i][j];
      PKS_UNROLL for (int t = 0; t < j; ++t) v -= L[i][t] * L[j][t];
      L[i][j] = v * inv;
    }
    PKS_UNROLL for (int i = 0; i < j; ++i) L[i][j] = R(0);
  }
  return ok;
}

// P = L L^T (symmetric), L lower triangular.
template <int N, typename R>
PKS_DEV void tril_gram(const R (&L)[N][N], R (&P)[N][N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = i; j < N; ++j) {
      R s = R(0);
      PKS_UNROLL for (int t = 0; t <= i; ++t) s += L[i][t] * L[j][t];
      P[i][j] = s;
      P[j][i] = s;
    }
}

// Packed lower triangles (the same N(N+1)/2 words as the symmetric blocks).
template <int N, typename R>
PKS_DEV void ld_tril(const R* __restrict__ base, size_t stride, size_t s, R (&L)[N][N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = 0; j < N; ++j) L[i][j] = j <= i ? base[sym_index<N>(j, i) * stride + s] : R(0);
}

template <int N, typename R>
PKS_DEV void st_tril(R* __restrict__ base, size_t stride, size_t s, const R (&L)[N][N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = 0; j <= i; ++j) base[sym_index<N>(j, i) * stride + s] = L[i][j];
}

template <int N, typename R, class Mv>
PKS_DEV void move_tril(const R (&L)[N][N], const Mv& mv, R (&O)[N][N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = 0; j < N; ++j) O[i][j] = j <= i ? mv(L[i][j]) : R(0);
}

// ---------------------------------------------------------------------------
// Filtering operator (eq. 15) on factors.
// ---------------------------------------------------------------------------
template <int N, typename R>
struct SqrtFilterElem {
  R A[N][N], b[N], U[N][N], eta[N], Z[N][N];
};
template <int N, typename R>
struct SqrtFilterCarry {
  R b[N], U[N][N];
};

template <int N, typename R, bool kIsolate = true>
struct SqrtFilterOp {
  // the scan ladders keep one copy of the operator instead of unrolling it
  static constexpr bool kCompact = true;
  using Elem = SqrtFilterElem<N, R>;
  using Carry = SqrtFilterCarry<N, R>;
  static constexpr int kS = sym_size<N>();
  static constexpr int kElemWords = N * N + 2 * N + 2 * kS;
  static constexpr int kCarryWords = N + kS;

  static PKS_DEV void load(const R* p, size_t st, size_t i, Elem& e) {
    ld_mat<N, N>(p, st, i, e.A);
    ld_vec<N>(p + N * N * st, st, i, e.b);
    ld_tril<N>(p + (N * N + N) * st, st, i, e.U);
    ld_vec<N>(p + (N * N + N + kS) * st, st, i, e.eta);
    ld_tril<N>(p + (N * N + 2 * N + kS) * st, st, i, e.Z);
  }
  static PKS_DEV void store(R* p, size_t st, size_t i, const Elem& e) {
    st_mat<N, N>(p, st, i, e.A);
    st_vec<N>(p + N * N * st, st, i, e.b);
    st_tril<N>(p + (N * N + N) * st, st, i, e.U);
    st_vec<N>(p + (N * N + N + kS) * st, st, i, e.eta);
    st_tril<N>(p + (N * N + 2 * N + kS) * st, st, i, e.Z);
  }
  static PKS_DEV void load(const R* p, size_t st, size_t i, Carry& c) {
    ld_vec<N>(p, st, i, c.b);
    ld_tril<N>(p + N * st, st, i, c.U);
  }
  static PKS_DEV void store(R* p, size_t st, size_t i, const Carry& c) {
    st_vec<N>(p, st, i, c.b);
    st_tril<N>(p + N * st, st, i, c.U);
  }
  template <class Mv>
  static PKS_DEV void move(const Elem& e, const Mv& mv, Elem& o) {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      o.b[i] = mv(e.b[i]);
      o.eta[i] = mv(e.eta[i]);
      PKS_UNROLL for (int j = 0; j < N; ++j) o.A[i][j] = mv(e.A[i][j]);
    }
    move_tril<N>(e.U, mv, o.U);
    move_tril<N>(e.Z, mv, o.Z);
  }
  static PKS_DEV void to_carry(const Elem& e, Carry& c) {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      c.b[i] = e.b[i];
      PKS_UNROLL for (int j = 0; j < N; ++j) c.U[i][j] = e.U[i][j];
    }
  }
  static PKS_DEV bool restarts(const R (&A)[N][N]) { return FilterOp<N, R, kIsolate>::restarts(A); }

  // Xi = tria([B, I]) for B = U^T Zj; W = U Xi^-T; V = Xi^-1 B Zj^T (V nullable work).
  static PKS_DEV void core(const R (&U)[N][N], const R (&Zj)[N][N], R (&B)[N][N], R (&W)[N][N]) {
    // B = U^T Zj  (U lower: U^T upper)
    PKS_UNROLL for (int i = 0; i < N; ++i)
      PKS_UNROLL for (int j = 0; j < N; ++j) {
        R s = R(0);
        PKS_UNROLL for (int t = (i > j ? i : j); t < N; ++t) s += U[t][i] * Zj[t][j];
        B[i][j] = s;
      }
    R X[N][2 * N], Xi[N][N];
    PKS_UNROLL for (int i = 0; i < N; ++i)
      PKS_UNROLL for (int j = 0; j < N; ++j) {
        X[i][j] = B[i][j];
        X[i][N + j] = R(i == j);
      }
    tria<N, 2 * N>(X, Xi);
    // W^T = Xi^-1 U^T
    R Wt[N][N];
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Wt[i][j] = U[j][i];
    tril_solve<N, N>(Xi, Wt);
    // B <- V = Xi^-1 B Zj^T
    R BZ[N][N];
    PKS_UNROLL for (int i = 0; i < N; ++i)
      PKS_UNROLL for (int j = 0; j < N; ++j) {
        R s = R(0);
        PKS_UNROLL for (int t = 0; t <= j; ++t) s += B[i][t] * Zj[j][t];
        BZ[i][j] = s;
      }
    tril_solve<N, N>(Xi, BZ);
    PKS_UNROLL for (int i = 0; i < N; ++i)
      PKS_UNROLL for (int j = 0; j < N; ++j) {
        W[i][j] = Wt[j][i];
      }
    // keep B^T Zj-free copy for Phi in the caller: B is overwritten only after use there
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) B[i][j] = BZ[i][j];
  }

  // bo = A_j (b + W (W^T eta_j - V b)) + b_j
  static PKS_DEV void mean_update(const R (&b)[N], const Elem& r, const R (&V)[N][N], const R (&W)[N][N],
                                  R (&bo)[N]) {
    R u[N], vb[N], t[N];
    mat_tvec<N, N>(W, r.eta, u);
    mat_vec<N, N>(V, b, vb);
    PKS_UNROLL for (int i = 0; i < N; ++i) u[i] -= vb[i];
    mat_vec<N, N>(W, u, t);
    PKS_UNROLL for (int i = 0; i < N; ++i) t[i] += b[i];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = r.b[i];
      PKS_UNROLL for (int k = 0; k < N; ++k) s += r.A[i][k] * t[k];
      bo[i] = s;
    }
  }

  // out = l (x) r
  static PKS_DEV void combine(const Elem& l, const Elem& r, Elem& o) {
    if (restarts(r.A)) {
      o = r;
      return;
    }
    // Xi22 = Zj Phi^-T with Phi = tria([B^T, I]), B = Ui^T Zj
    R X22[N][N];
    {
      R X[N][2 * N], Phi[N][N];
      PKS_UNROLL for (int i = 0; i < N; ++i)
        PKS_UNROLL for (int j = 0; j < N; ++j) {
          R s = R(0);   // (B^T)[i][j] = B[j][i] = sum_t U[t][j] Z[t][i]
          PKS_UNROLL for (int t = (i > j ? i : j); t < N; ++t) s += l.U[t][j] * r.Z[t][i];
          X[i][j] = s;
          X[i][N + j] = R(i == j);
        }
      tria<N, 2 * N>(X, Phi);
      // X22^T = Phi^-1 Zj^T
      R T[N][N];
      PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) T[i][j] = r.Z[j][i];
      tril_solve<N, N>(Phi, T);
      PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) X22[i][j] = T[j][i];
    }
    R V[N][N], W[N][N];
    core(l.U, r.Z, V, W);
    // A_ij = A_j (A_i - W (V A_i))
    {
      R VA[N][N], T[N][N];
      mat_mul<N, N, N>(V, l.A, VA);
      mat_mul<N, N, N>(W, VA, T);
      PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) T[i][j] = l.A[i][j] - T[i][j];
      mat_mul<N, N, N>(r.A, T, o.A);
    }
    // b_ij = A_j (b_i + W (W^T eta_j - V b_i)) + b_j: (I + C_i J_j)^-1 (b_i + C_i eta_j)
    // = (I - W V) b_i + W W^T eta_j, with no large intermediate to cancel
    mean_update(l.b, r, V, W, o.b);
    // eta_ij = A_i^T (s - V^T (W^T s)) + eta_i,  s = eta_j - Z_j (Z_j^T b_i)
    {
      R z[N], s[N], ws[N], vw[N];
      mat_tvec<N, N>(r.Z, l.b, z);
      mat_vec<N, N>(r.Z, z, s);
      PKS_UNROLL for (int i = 0; i < N; ++i) s[i] = r.eta[i] - s[i];
      mat_tvec<N, N>(W, s, ws);
      mat_tvec<N, N>(V, ws, vw);
      PKS_UNROLL for (int i = 0; i < N; ++i) s[i] -= vw[i];
      mat_tvec<N, N>(l.A, s, z);
      PKS_UNROLL for (int i = 0; i < N; ++i) o.eta[i] = z[i] + l.eta[i];
    }
    // U_ij = tria([A_j W, U_j])
    {
      R AW[N][N], X[N][2 * N];
      mat_mul<N, N, N>(r.A, W, AW);
      hcat<N, N, N>(AW, r.U, X);
      tria<N, 2 * N>(X, o.U);
    }
    // Z_ij = tria([A_i^T Xi22, Z_i])
    {
      R AX[N][N], X[N][2 * N];
      PKS_UNROLL for (int i = 0; i < N; ++i)
        PKS_UNROLL for (int j = 0; j < N; ++j) {
          R s = R(0);
          PKS_UNROLL for (int t = 0; t < N; ++t) s += l.A[t][i] * X22[t][j];
          AX[i][j] = s;
        }
      hcat<N, N, N>(AX, l.Z, X);
      tria<N, 2 * N>(X, o.Z);
    }
  }

  // out = c (x) r for a carry c
  static PKS_DEV void apply(const Carry& c, const Elem& r, Carry& o) {
    if (restarts(r.A)) {
      PKS_UNROLL for (int i = 0; i < N; ++i) {
        o.b[i] = r.b[i];
        PKS_UNROLL for (int j = 0; j < N; ++j) o.U[i][j] = r.U[i][j];
      }
      return;
    }
    R V[N][N], W[N][N];
    core(c.U, r.Z, V, W);
    mean_update(c.b, r, V, W, o.b);
    R AW[N][N], X[N][2 * N];
    mat_mul<N, N, N>(r.A, W, AW);
    hcat<N, N, N>(AW, r.U, X);
    tria<N, 2 * N>(X, o.U);
  }
};

// ---------------------------------------------------------------------------
// Smoothing operator (eq. 19) on factors.
// ---------------------------------------------------------------------------
template <int N, typename R>
struct SqrtSmootherElem {
  R E[N][N], g[N], D[N][N];
};
template <int N, typename R>
struct SqrtSmootherCarry {
  R g[N], D[N][N];
};

template <int N, typename R, bool kIsolate = true>
struct SqrtSmootherOp {
  // the scan ladders keep one copy of the operator instead of unrolling it
  static constexpr bool kCompact = true;
  using Elem = SqrtSmootherElem<N, R>;
  using Carry = SqrtSmootherCarry<N, R>;
  static constexpr int kS = sym_size<N>();
  static constexpr int kElemWords = N * N + N + kS;
  static constexpr int kCarryWords = N + kS;

  static PKS_DEV void load(const R* p, size_t st, size_t i, Elem& e) {
    ld_mat<N, N>(p, st, i, e.E);
    ld_vec<N>(p + N * N * st, st, i, e.g);
    ld_tril<N>(p + (N * N + N) * st, st, i, e.D);
  }
  static PKS_DEV void store(R* p, size_t st, size_t i, const Elem& e) {
    st_mat<N, N>(p, st, i, e.E);
    st_vec<N>(p + N * N * st, st, i, e.g);
    st_tril<N>(p + (N * N + N) * st, st, i, e.D);
  }
  static PKS_DEV void load(const R* p, size_t st, size_t i, Carry& c) {
    ld_vec<N>(p, st, i, c.g);
    ld_tril<N>(p + N * st, st, i, c.D);
  }
  static PKS_DEV void store(R* p, size_t st, size_t i, const Carry& c) {
    st_vec<N>(p, st, i, c.g);
    st_tril<N>(p + N * st, st, i, c.D);
  }
  template <class Mv>
  static PKS_DEV void move(const Elem& e, const Mv& mv, Elem& o) {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      o.g[i] = mv(e.g[i]);
      PKS_UNROLL for (int j = 0; j < N; ++j) o.E[i][j] = mv(e.E[i][j]);
    }
    move_tril<N>(e.D, mv, o.D);
  }
  static PKS_DEV void to_carry(const Elem& e, Carry& c) {
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      c.g[i] = e.g[i];
      PKS_UNROLL for (int j = 0; j < N; ++j) c.D[i][j] = e.D[i][j];
    }
  }
  static PKS_DEV bool restarts(const R (&E)[N][N]) { return SmootherOp<N, R, kIsolate>::restarts(E); }

  // Scan order: x precedes y in the scan (x is the later slot); out = y (x) x.
  static PKS_DEV void combine(const Elem& x, const Elem& y, Elem& o) {
    if (restarts(y.E)) {
      PKS_UNROLL for (int i = 0; i < N; ++i) {
        o.g[i] = y.g[i];
        PKS_UNROLL for (int j = 0; j < N; ++j) {
          o.E[i][j] = R(0);
          o.D[i][j] = y.D[i][j];
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
    R ED[N][N], X[N][2 * N];
    mat_mul<N, N, N>(y.E, x.D, ED);
    hcat<N, N, N>(ED, y.D, X);
    tria<N, 2 * N>(X, o.D);
  }
  static PKS_DEV void apply(const Carry& c, const Elem& y, Carry& o) {
    if (restarts(y.E)) {
      PKS_UNROLL for (int i = 0; i < N; ++i) {
        o.g[i] = y.g[i];
        PKS_UNROLL for (int j = 0; j < N; ++j) o.D[i][j] = y.D[i][j];
      }
      return;
    }
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = y.g[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) s += y.E[i][t] * c.g[t];
      o.g[i] = s;
    }
    R ED[N][N], X[N][2 * N];
    mat_mul<N, N, N>(y.E, c.D, ED);
    hcat<N, N, N>(ED, y.D, X);
    tria<N, 2 * N>(X, o.D);
  }
};

// ---------------------------------------------------------------------------
// Elements.
// ---------------------------------------------------------------------------
// Filtering element (eq. 13-14) in factor form from the surrogate transition
// (F, c, Q') into the slot and the measurement model (H, d, R', ytil) at it.
// With Uq = chol Q', Ur = chol R':
//   tria([[Ur, H Uq], [0, Uq]]) = [[S1, 0], [K1, U]]
// where S1 S1^T = S = H Q' H^T + R', K1 = Q' H^T S1^-T and U U^T = Q' - K S K^T
// = C; the gain is K = K1 S1^-1.  Then A = F - K H F, b = c + K (y - H c - d),
// and with Y = S1^-1 H F, w = S1^-1 (y - H c - d): J = Y^T Y, eta = Y^T w, so
// Z = tria([Y^T, 0]).  Returns false if Q' is not positive semi-definite or
// R' not positive definite.
template <int N, int P, typename R>
PKS_DEV bool sqrt_filter_element(const R (&F)[N][N], const R (&c)[N], const R (&Qp)[N][N], const R (&H)[P][N],
                                 const R (&d)[P], const R (&Rp)[P][P], const R (&y)[P], R (&A)[N][N], R (&b)[N],
                                 R (&U)[N][N], R (&eta)[N], R (&Z)[N][N]) {
  constexpr int M = P + N;
  R Uq[N][N], Ur[P][P];
  bool ok = chol_lower_psd<N>(Qp, Uq);
  ok = chol_lower<P>(Rp, Ur) && ok;
  R X[M][M];
  PKS_UNROLL for (int i = 0; i < P; ++i) {
    PKS_UNROLL for (int j = 0; j < P; ++j) X[i][j] = Ur[i][j];
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      R s = R(0);
      PKS_UNROLL for (int t = j; t < N; ++t) s += H[i][t] * Uq[t][j];
      X[i][P + j] = s;
    }
  }
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    PKS_UNROLL for (int j = 0; j < P; ++j) X[P + i][j] = R(0);
    PKS_UNROLL for (int j = 0; j < N; ++j) X[P + i][P + j] = Uq[i][j];
  }
  R T[M][M];
  tria<M, M>(X, T);
  R S1[P][P];
  PKS_UNROLL for (int i = 0; i < P; ++i) PKS_UNROLL for (int j = 0; j < P; ++j) S1[i][j] = T[i][j];
  PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) U[i][j] = T[P + i][P + j];
  // G = (S1^-1 (K1)^T)^T = K (N x P): solve S1 Kt = K1^T
  R Kt[P][N];
  PKS_UNROLL for (int i = 0; i < P; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Kt[i][j] = T[P + j][i];
  tril_tsolve<P, N>(S1, Kt);       // K^T = S1^-T K1^T
  // HF, innovation
  R HF[P][N], e[P];
  mat_mul<P, N, N>(H, F, HF);
  PKS_UNROLL for (int i = 0; i < P; ++i) {
    R s = y[i] - d[i];
    PKS_UNROLL for (int t = 0; t < N; ++t) s -= H[i][t] * c[t];
    e[i] = s;
  }
  // A = F - K HF, b = c + K e
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R s = c[i];
    PKS_UNROLL for (int k = 0; k < P; ++k) s += Kt[k][i] * e[k];
    b[i] = s;
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      R a = F[i][j];
      PKS_UNROLL for (int k = 0; k < P; ++k) a -= Kt[k][i] * HF[k][j];
      A[i][j] = a;
    }
  }
  // Y = S1^-1 HF, w = S1^-1 e
  tril_solve<P, N>(S1, HF);
  R w[P][1];
  PKS_UNROLL for (int i = 0; i < P; ++i) w[i][0] = e[i];
  tril_solve<P, 1>(S1, w);
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R s = R(0);
    PKS_UNROLL for (int k = 0; k < P; ++k) s += HF[k][i] * w[k][0];
    eta[i] = s;
  }
  R Yt[N][N];
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = 0; j < N; ++j) Yt[i][j] = j < P ? HF[j][i] : R(0);
  tria<N, N>(Yt, Z);
  return ok;
}

// Smoothing element (eq. 17) in factor form from the filtered x*, P* = U U^T
// and the surrogate transition (F, c, Q') out of the slot.  With Uq = chol Q',
//   tria([[F U, Uq], [U, 0]]) = [[Phi, 0], [G, D]]
// gives Phi Phi^T = F P* F^T + Q', G Phi^T = P* F^T and D D^T = P* - G G^T =
// P* - E F P* = L (the Schur complement, obtained by orthogonal reductions
// only), so E = G Phi^-1, g = x* - E (F x* + c).  Returns false if Q' is not
// positive semi-definite.
template <int N, typename R>
PKS_DEV bool sqrt_smoother_element(const R (&x)[N], const R (&U)[N][N], const R (&F)[N][N], const R (&c)[N],
                                   const R (&Qp)[N][N], R (&E)[N][N], R (&g)[N], R (&D)[N][N]) {
  R Uq[N][N];
  const bool ok = chol_lower_psd<N>(Qp, Uq);
  R X[2 * N][2 * N];
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      R s = R(0);
      PKS_UNROLL for (int t = j; t < N; ++t) s += F[i][t] * U[t][j];
      X[i][j] = s;
      X[i][N + j] = Uq[i][j];
      X[N + i][j] = U[i][j];
      X[N + i][N + j] = R(0);
    }
  R T[2 * N][2 * N];
  tria<2 * N, 2 * N>(X, T);
  // E^T = Phi^-T G^T
  R Et[N][N], Phi[N][N];
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      Phi[i][j] = T[i][j];
      Et[i][j] = T[N + j][i];
      D[i][j] = T[N + i][N + j];
    }
  tril_tsolve<N, N>(Phi, Et);
  PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) E[i][j] = Et[j][i];
  // g = x - E (F x + c)
  R fx[N];
  mat_vec<N, N>(F, x, fx);
  PKS_UNROLL for (int i = 0; i < N; ++i) fx[i] += c[i];
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R s = x[i];
    PKS_UNROLL for (int t = 0; t < N; ++t) s -= E[i][t] * fx[t];
    g[i] = s;
  }
  return ok;
}

}  // namespace pks
