// Register-resident small dense linear algebra for one lane.
//
// Every routine is fully unrolled over compile-time dimensions so that the
// operands stay in VGPRs (no dynamic indexing, hence no scratch).  Symmetric
// positive-definite systems are solved through Cholesky factors; nothing here
// pivots, so control flow is uniform across a wavefront.
#pragma once

#include <hip/hip_runtime.h>

namespace pks {

#define PKS_DEV __device__ __forceinline__
#define PKS_HD __host__ __device__ __forceinline__
#define PKS_UNROLL _Pragma("unroll")

// Number of entries of an upper-packed symmetric N x N matrix.
template <int N>
constexpr int sym_size() { return N * (N + 1) / 2; }

// Row-major upper-packed index of (i, j), i <= j.
template <int N>
constexpr int sym_index(int i, int j) {
  return i <= j ? i * N - i * (i - 1) / 2 + (j - i) : j * N - j * (j - 1) / 2 + (i - j);
}

// 1/sqrt(x) and 1/x from the hardware estimates refined by two Newton steps
// (each step squares the relative error), instead of the long IEEE
// square-root / divide sequences: these sit on the dependency chain of every
// Cholesky factorisation in the scans.
PKS_DEV double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  PKS_UNROLL for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
PKS_DEV float rsqrt_nr(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  const float e = fmaf(-x * y, y, 1.0f);
  return fmaf(0.5f * y, e, y);
}
PKS_DEV double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  PKS_UNROLL for (int it = 0; it < 2; ++it) {
    const double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
  }
  return r;
}
PKS_DEV float rcp_nr(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}

// ---------------------------------------------------------------------------
// Cholesky: A = L L^T (lower L), in place on a full symmetric array.  The
// diagonal of the result holds 1/L_jj (reciprocals are what the solves use);
// if diag is given it receives L_jj itself.  Returns false if a pivot is not
// positive (callers turn that into NaN outputs).
// ---------------------------------------------------------------------------
template <int N, typename R>
PKS_DEV bool chol_inplace(R (&A)[N][N], R* diag = nullptr) {
  bool ok = true;
  PKS_UNROLL for (int j = 0; j < N; ++j) {
    R s = A[j][j];
    PKS_UNROLL for (int t = 0; t < j; ++t) s -= A[j][t] * A[j][t];
    ok = ok && (s > R(0));
    const R inv = rsqrt_nr(s);
    if (diag) diag[j] = s * inv;
    PKS_UNROLL for (int i = j + 1; i < N; ++i) {
      R v = A[i][j];
      PKS_UNROLL for (int t = 0; t < j; ++t) v -= A[i][t] * A[j][t];
      A[i][j] = v * inv;
    }
    A[j][j] = inv;
  }
  return ok;
}

// Solve L z = b for M right-hand sides stored as columns of B (N x M), in place.
// L comes from chol_inplace (reciprocal diagonal).
template <int N, int M, typename R>
PKS_DEV void chol_fwd(const R (&L)[N][N], R (&B)[N][M]) {
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    PKS_UNROLL for (int c = 0; c < M; ++c) {
      R s = B[i][c];
      PKS_UNROLL for (int t = 0; t < i; ++t) s -= L[i][t] * B[t][c];
      B[i][c] = s * L[i][i];
    }
  }
}

// Solve L^T x = z for M right-hand sides (columns of B), in place.
template <int N, int M, typename R>
PKS_DEV void chol_bwd(const R (&L)[N][N], R (&B)[N][M]) {
  PKS_UNROLL for (int i = N - 1; i >= 0; --i) {
    PKS_UNROLL for (int c = 0; c < M; ++c) {
      R s = B[i][c];
      PKS_UNROLL for (int t = i + 1; t < N; ++t) s -= L[t][i] * B[t][c];
      B[i][c] = s * L[i][i];
    }
  }
}

template <int N, typename R>
PKS_DEV void chol_fwd_vec(const R (&L)[N][N], R (&b)[N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R s = b[i];
    PKS_UNROLL for (int t = 0; t < i; ++t) s -= L[i][t] * b[t];
    b[i] = s * L[i][i];
  }
}

// ---------------------------------------------------------------------------
// Products.
// ---------------------------------------------------------------------------
// C = A B
template <int M, int K, int N, typename R>
PKS_DEV void mat_mul(const R (&A)[M][K], const R (&B)[K][N], R (&C)[M][N]) {
  PKS_UNROLL for (int i = 0; i < M; ++i)
    PKS_UNROLL for (int j = 0; j < N; ++j) {
      R s = A[i][0] * B[0][j];
      PKS_UNROLL for (int t = 1; t < K; ++t) s += A[i][t] * B[t][j];
      C[i][j] = s;
    }
}

// y = A x
template <int M, int K, typename R>
PKS_DEV void mat_vec(const R (&A)[M][K], const R (&x)[K], R (&y)[M]) {
  PKS_UNROLL for (int i = 0; i < M; ++i) {
    R s = A[i][0] * x[0];
    PKS_UNROLL for (int t = 1; t < K; ++t) s += A[i][t] * x[t];
    y[i] = s;
  }
}

// y = A^T x, A is (K x M)
template <int K, int M, typename R>
PKS_DEV void mat_tvec(const R (&A)[K][M], const R (&x)[K], R (&y)[M]) {
  PKS_UNROLL for (int i = 0; i < M; ++i) {
    R s = A[0][i] * x[0];
    PKS_UNROLL for (int t = 1; t < K; ++t) s += A[t][i] * x[t];
    y[i] = s;
  }
}

// S = A B A^T + Cadd with S symmetric (upper triangle computed, mirrored).
// A is (M x K), B is (K x K) symmetric.
template <int M, int K, typename R>
PKS_DEV void sandwich_add(const R (&A)[M][K], const R (&B)[K][K], const R (&Cadd)[M][M],
                          R (&S)[M][M]) {
  R AB[M][K];
  mat_mul<M, K, K>(A, B, AB);
  PKS_UNROLL for (int i = 0; i < M; ++i)
    PKS_UNROLL for (int j = i; j < M; ++j) {
      R s = Cadd[i][j];
      PKS_UNROLL for (int t = 0; t < K; ++t) s += AB[i][t] * A[j][t];
      S[i][j] = s;
      S[j][i] = s;
    }
}

// S = A^T B A + Cadd, symmetric; A is (K x M), B (K x K) symmetric.
template <int K, int M, typename R>
PKS_DEV void tsandwich_add(const R (&A)[K][M], const R (&B)[K][K], const R (&Cadd)[M][M],
                           R (&S)[M][M]) {
  R BA[K][M];
  mat_mul<K, K, M>(B, A, BA);
  PKS_UNROLL for (int i = 0; i < M; ++i)
    PKS_UNROLL for (int j = i; j < M; ++j) {
      R s = Cadd[i][j];
      PKS_UNROLL for (int t = 0; t < K; ++t) s += A[t][i] * BA[t][j];
      S[i][j] = s;
      S[j][i] = s;
    }
}

// G = Z^T Z (symmetric), Z is (K x M).
template <int K, int M, typename R>
PKS_DEV void gram(const R (&Z)[K][M], R (&G)[M][M]) {
  PKS_UNROLL for (int i = 0; i < M; ++i)
    PKS_UNROLL for (int j = i; j < M; ++j) {
      R s = Z[0][i] * Z[0][j];
      PKS_UNROLL for (int t = 1; t < K; ++t) s += Z[t][i] * Z[t][j];
      G[i][j] = s;
      G[j][i] = s;
    }
}

template <int N, typename R>
PKS_DEV void set_zero(R (&A)[N][N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) A[i][j] = R(0);
}

template <int N, typename R>
PKS_DEV void set_zero(R (&a)[N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i) a[i] = R(0);
}

template <typename R> PKS_DEV R quiet_nan();
template <> PKS_DEV double quiet_nan<double>() { return __builtin_nan(""); }
template <> PKS_DEV float quiet_nan<float>() { return __builtin_nanf(""); }

// ---------------------------------------------------------------------------
// Strided structure-of-arrays access: entry e of slot s lives at base[e*stride + s].
// ---------------------------------------------------------------------------
template <int N, typename R>
PKS_DEV void ld_vec(const R* __restrict__ base, size_t stride, size_t s, R (&v)[N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i) v[i] = base[i * stride + s];
}

template <int N, typename R>
PKS_DEV void st_vec(R* __restrict__ base, size_t stride, size_t s, const R (&v)[N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i) base[i * stride + s] = v[i];
}

template <int M, int N, typename R>
PKS_DEV void ld_mat(const R* __restrict__ base, size_t stride, size_t s, R (&A)[M][N]) {
  PKS_UNROLL for (int i = 0; i < M; ++i)
    PKS_UNROLL for (int j = 0; j < N; ++j) A[i][j] = base[(i * N + j) * stride + s];
}

template <int M, int N, typename R>
PKS_DEV void st_mat(R* __restrict__ base, size_t stride, size_t s, const R (&A)[M][N]) {
  PKS_UNROLL for (int i = 0; i < M; ++i)
    PKS_UNROLL for (int j = 0; j < N; ++j) base[(i * N + j) * stride + s] = A[i][j];
}

template <int N, typename R>
PKS_DEV void ld_sym(const R* __restrict__ base, size_t stride, size_t s, R (&A)[N][N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = i; j < N; ++j) {
      const R v = base[sym_index<N>(i, j) * stride + s];
      A[i][j] = v;
      A[j][i] = v;
    }
}

template <int N, typename R>
PKS_DEV void st_sym(R* __restrict__ base, size_t stride, size_t s, const R (&A)[N][N]) {
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = i; j < N; ++j) base[sym_index<N>(i, j) * stride + s] = A[i][j];
}

}  // namespace pks
