// Wavefront-cooperative form of the method for larger states (n = 20): one
// 64-lane workgroup owns one element at a time, with its N x N matrices in
// LDS, and the scans run as a hierarchy of chunk folds (Section 4, eq. 15 and
// eq. 19 evaluated as in operators.hpp; elements as in elements.hpp).
//
// HBM records are slot-major (all words of one slot contiguous), so a wave
// reads or writes one record with contiguous lanes.  Symmetric matrices are
// stored upper-packed (sym_index order) in HBM and full in LDS.
#pragma once

#include "elements.hpp"
#include "slot_kernels.hpp"

namespace pks {
namespace dn {

constexpr int kWave = 64;

template <int N>
constexpr int ld() { return N + 1; }           // LDS row length (odd: spreads banks)
template <int N>
constexpr int mat_words() { return N * ld<N>(); }

PKS_DEV int lane() { return int(threadIdx.x); }
PKS_DEV void wsync() { __syncthreads(); }     // workgroups are a single wave

// ---------------------------------------------------------------------------
// Wave-wide matrix routines on LDS operands (leading dimension ld<LDN>()).
// Each ends with a barrier, so its results are visible to every lane.
// ---------------------------------------------------------------------------

typedef double f64x4 __attribute__((ext_vector_type(4)));

// The VALU form of mm below: each lane computes a 2 x 4 block of C, so every
// LDS word it loads feeds two or four multiply-adds.
template <int LDN, int M, int K, int NC, bool TA, bool TB, typename R>
PKS_DEV void mm_valu(const R* A, const R* B, const R* C0, R sgn, R* C) {
  constexpr int L = ld<LDN>();
  constexpr int TR = 2, TC = 4;
  constexpr int MR = (M + TR - 1) / TR, MC = (NC + TC - 1) / TC;
  for (int t = lane(); t < MR * MC; t += kWave) {
    const int i0 = (t / MC) * TR, j0 = (t % MC) * TC;
    R acc[TR][TC];
    PKS_UNROLL for (int r = 0; r < TR; ++r) PKS_UNROLL for (int c = 0; c < TC; ++c) acc[r][c] = R(0);
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
      R a[TR], b[TC];
      PKS_UNROLL for (int r = 0; r < TR; ++r) {
        const int i = i0 + r;
        a[r] = (M % TR == 0 || i < M) ? (TA ? A[k * L + i] : A[i * L + k]) : R(0);
      }
      PKS_UNROLL for (int c = 0; c < TC; ++c) {
        const int j = j0 + c;
        b[c] = (NC % TC == 0 || j < NC) ? (TB ? B[j * L + k] : B[k * L + j]) : R(0);
      }
      PKS_UNROLL for (int r = 0; r < TR; ++r) PKS_UNROLL for (int c = 0; c < TC; ++c)
        acc[r][c] = fma(a[r], b[c], acc[r][c]);
    }
    PKS_UNROLL for (int r = 0; r < TR; ++r) PKS_UNROLL for (int c = 0; c < TC; ++c) {
      const int i = i0 + r, j = j0 + c;
      if ((M % TR == 0 || i < M) && (NC % TC == 0 || j < NC))
        C[i * L + j] = (C0 ? C0[i * L + j] : R(0)) + sgn * acc[r][c];
    }
  }
  wsync();
}

// C = C0 + sgn * op(A) op(B), op(A) M x K, op(B) K x NC.  C may alias C0 but
// not A or B.  C0 may be null (zero).  FP64 20 x 20 x 20 (the full-state
// blocks): v_mfma_f64_16x16x4f64 on the product padded to 32 x 32, 2 x 2
// output tiles, 5 steps of 4 along the reduction; lane l feeds A[l % 16][l /
// 16] and B[l / 16][l % 16] and receives D[4 q + l / 16][l % 16], q = 0..3.
// Two LDS words per 2048 flops against six per eight multiply-adds on the
// VALU (mm_valu, measured against it by libdense_probe.so).  Other shapes and
// FP32: mm_valu.
template <int LDN, int M, int K, int NC, bool TA, bool TB, typename R>
PKS_DEV void mm(const R* A, const R* B, const R* C0, R sgn, R* C) {
  constexpr int L = ld<LDN>();
  if constexpr (sizeof(R) == 8 && M == 20 && K == 20 && NC == 20) {
    // Every LDS read is unconditional and issued before the first MFMA: rows
    // and columns past 19 of the padded operands read row or column 19 and
    // are replaced by zero with a select, and result elements past 19 (and
    // their C0 reads) go to column 20 of the rows, the unused padding of the
    // LDS layout, instead of being skipped behind branches.
    const int r = lane() & 15, kq = lane() >> 4;
    double av[5][2], bv[5][2];
    PKS_UNROLL for (int ks = 0; ks < 5; ++ks) {
      const int k = 4 * ks + kq;   // < 20
      PKS_UNROLL for (int t = 0; t < 2; ++t) {
        const int i = 16 * t + r, ic = i < 20 ? i : 19;
        const double a = double(TA ? A[k * L + ic] : A[ic * L + k]);
        const double b = double(TB ? B[ic * L + k] : B[k * L + ic]);
        av[ks][t] = i < 20 ? a : 0.0;
        bv[ks][t] = i < 20 ? b : 0.0;
      }
    }
    int at[2][2][4];
    R c0[2][2][4];
    PKS_UNROLL for (int ti = 0; ti < 2; ++ti)
      PKS_UNROLL for (int tj = 0; tj < 2; ++tj)
        PKS_UNROLL for (int q = 0; q < 4; ++q) {
          const int i = 16 * ti + 4 * q + kq, j = 16 * tj + r;
          at[ti][tj][q] = (i < 20 && j < 20) ? i * L + j : (i < 20 ? i : i - 20) * L + 20;
          c0[ti][tj][q] = C0 ? C0[at[ti][tj][q]] : R(0);
        }
    f64x4 acc[2][2];
    PKS_UNROLL for (int i = 0; i < 2; ++i) PKS_UNROLL for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    PKS_UNROLL for (int ks = 0; ks < 5; ++ks)
      PKS_UNROLL for (int ti = 0; ti < 2; ++ti)
        PKS_UNROLL for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks][ti], bv[ks][tj], acc[ti][tj], 0, 0, 0);
    PKS_UNROLL for (int ti = 0; ti < 2; ++ti)
      PKS_UNROLL for (int tj = 0; tj < 2; ++tj)
        PKS_UNROLL for (int q = 0; q < 4; ++q) C[at[ti][tj][q]] = c0[ti][tj][q] + sgn * R(acc[ti][tj][q]);
    wsync();
    return;
  }
  mm_valu<LDN, M, K, NC, TA, TB, R>(A, B, C0, sgn, C);
}

// y = y0 + sgn * op(A) x, op(A) M x K.  y may alias y0 but not x.
template <int LDN, int M, int K, bool TA, typename R>
PKS_DEV void mv(const R* A, const R* x, const R* y0, R sgn, R* y) {
  constexpr int L = ld<LDN>();
  for (int i = lane(); i < M; i += kWave) {
    R s = R(0);
    PKS_UNROLL for (int k = 0; k < K; ++k) s = fma(TA ? A[k * L + i] : A[i * L + k], x[k], s);
    y[i] = (y0 ? y0[i] : R(0)) + sgn * s;
  }
  wsync();
}

// Value of x in lane `src` (uniform), as a double.
PKS_DEV double lane_value(double x, int src) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(int(v & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane(int(v >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// In-place lower Cholesky factor (true diagonal); the upper triangle is
// cleared.  *ok (LDS) is cleared when a pivot is not positive; the factor then
// holds NaN, which reaches the convergence statistic.  Lane i keeps row i in
// registers; column j takes the finished entries of row j from lane j with
// cross-lane reads, so the whole factorisation touches LDS twice.
template <int LDN, int N, typename R>
PKS_DEV void chol(R* A, int* ok) {
  static_assert(N <= kWave, "one row per lane");
  constexpr int L = ld<LDN>();
  const int i = lane();
  R row[N];
  PKS_UNROLL for (int k = 0; k < N; ++k) row[k] = i < N ? A[i * L + k] : R(0);
  bool good = true;
  PKS_UNROLL for (int j = 0; j < N; ++j) {
    R s0 = row[j], s1 = R(0);
    PKS_UNROLL for (int t = 0; t < j; ++t) {
      const R ljt = lane_value(row[t], j);
      if (t & 1) s1 = fma(-row[t], ljt, s1);
      else s0 = fma(-row[t], ljt, s0);
    }
    const R s = s0 + s1;
    const R d = lane_value(s, j);               // pivot of column j
    good = good && d > R(0);
    const R sd = sqrt(d);
    row[j] = i == j ? sd : (i > j ? s / sd : R(0));
  }
  if (i < N) {
    PKS_UNROLL for (int k = 0; k < N; ++k) A[i * L + k] = k <= i ? row[k] : R(0);
  }
  if (i == 0 && !good) *ok = 0;
  wsync();
}

// B <- Lc^-1 B (forward substitution), Lc N x N lower, B N x NC; lane per
// column, the column kept in registers.
template <int LDN, int N, int NC, typename R>
PKS_DEV void fwd(const R* Lc, R* B) {
  constexpr int L = ld<LDN>();
  for (int c = lane(); c < NC; c += kWave) {
    R x[N];
    PKS_UNROLL for (int i = 0; i < N; ++i) x[i] = B[i * L + c];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = x[i];
      PKS_UNROLL for (int t = 0; t < i; ++t) s = fma(-Lc[i * L + t], x[t], s);
      x[i] = s / Lc[i * L + i];
    }
    PKS_UNROLL for (int i = 0; i < N; ++i) B[i * L + c] = x[i];
  }
  wsync();
}

// B <- Lc^-T B (back substitution).
template <int LDN, int N, int NC, typename R>
PKS_DEV void bwd(const R* Lc, R* B) {
  constexpr int L = ld<LDN>();
  for (int c = lane(); c < NC; c += kWave) {
    R x[N];
    PKS_UNROLL for (int i = 0; i < N; ++i) x[i] = B[i * L + c];
    PKS_UNROLL for (int i = N - 1; i >= 0; --i) {
      R s = x[i];
      PKS_UNROLL for (int t = i + 1; t < N; ++t) s = fma(-Lc[t * L + i], x[t], s);
      x[i] = s / Lc[i * L + i];
    }
    PKS_UNROLL for (int i = 0; i < N; ++i) B[i * L + c] = x[i];
  }
  wsync();
}

// x <- Lc^-1 x for one vector (lane 0, in registers).
template <int LDN, int N, typename R>
PKS_DEV void fwd_vec(const R* Lc, R* x) {
  constexpr int L = ld<LDN>();
  if (lane() == 0) {
    R y[N];
    PKS_UNROLL for (int i = 0; i < N; ++i) y[i] = x[i];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R s = y[i];
      PKS_UNROLL for (int t = 0; t < i; ++t) s = fma(-Lc[i * L + t], y[t], s);
      y[i] = s / Lc[i * L + i];
    }
    PKS_UNROLL for (int i = 0; i < N; ++i) x[i] = y[i];
  }
  wsync();
}

// A <- (A + A^T) / 2
template <int LDN, int N, typename R>
PKS_DEV void symmetrize(R* A) {
  // all reads issued before the first store (one LDS latency, not one per pass);
  // each pair (i < j) belongs to one lane
  constexpr int L = ld<LDN>();
  constexpr int T = N * N, RN = (T + kWave - 1) / kWave;
  R v[RN];
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    const int i = e / N, j = e - i * N;
    v[r] = (e < T && j > i) ? R(0.5) * (A[i * L + j] + A[j * L + i]) : R(0);
  }
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    const int i = e / N, j = e - i * N;
    if (e < T && j > i) {
      A[i * L + j] = v[r];
      A[j * L + i] = v[r];
    }
  }
  wsync();
}

template <int LDN, int M, int NC, bool TR, typename R>
PKS_DEV void copy(const R* A, R* B) {   // B = op(A), M x NC
  // all reads issued before the first store, as in symmetrize
  constexpr int L = ld<LDN>();
  constexpr int T = M * NC, RN = (T + kWave - 1) / kWave;
  R v[RN];
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    const int i = e / NC, j = e - i * NC;
    v[r] = e < T ? (TR ? A[j * L + i] : A[i * L + j]) : R(0);
  }
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    const int i = e / NC, j = e - i * NC;
    if (e < T) B[i * L + j] = v[r];
  }
  wsync();
}

template <int LDN, int M, int NC, typename R>
PKS_DEV void zero(R* A) {
  constexpr int L = ld<LDN>();
  for (int e = lane(); e < M * NC; e += kWave) A[(e / NC) * L + e % NC] = R(0);
  wsync();
}

template <int N, typename R>
PKS_DEV void vcopy(const R* x, R* y) {
  for (int i = lane(); i < N; i += kWave) y[i] = x[i];
  wsync();
}

// --- HBM <-> LDS ------------------------------------------------------------
// The element type in HBM (RG) may differ from the one in LDS (R): the FP32
// engine's linearisation works in FP64 on its FP32 records.
template <int LDN, int M, int NC, typename RG, typename R>
PKS_DEV void ld_full(const RG* g, R* A) {
  // all global loads are issued before the first LDS store (fixed trip
  // counts), so one record costs one memory latency, not one per pass
  constexpr int L = ld<LDN>();
  constexpr int T = M * NC, RN = (T + kWave - 1) / kWave;
  R v[RN];
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    v[r] = e < T ? R(g[e]) : R(0);
  }
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    if (e < T) A[(e / NC) * L + e % NC] = v[r];
  }
}
// A += g (row-major M x NC in HBM), loads issued first as in ld_full
template <int LDN, int M, int NC, typename RG, typename R>
PKS_DEV void add_full(const RG* g, R* A) {
  constexpr int L = ld<LDN>();
  constexpr int T = M * NC, RN = (T + kWave - 1) / kWave;
  R v[RN];
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    v[r] = e < T ? R(g[e]) : R(0);
  }
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    if (e < T) A[(e / NC) * L + e % NC] += v[r];
  }
}
template <int LDN, int M, int NC, typename R, typename RG>
PKS_DEV void st_full(const R* A, RG* g) {
  constexpr int L = ld<LDN>();
  for (int e = lane(); e < M * NC; e += kWave) g[e] = RG(A[(e / NC) * L + e % NC]);
}
template <int LDN, int N, typename RG, typename R>
PKS_DEV void ld_symm(const RG* g, R* A) {
  constexpr int L = ld<LDN>();
  constexpr int T = N * N, RN = (T + kWave - 1) / kWave;
  R v[RN];
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    const int i = e / N, j = e - i * N;
    v[r] = e < T ? R(g[sym_index<N>(i, j)]) : R(0);
  }
  PKS_UNROLL for (int r = 0; r < RN; ++r) {
    const int e = r * kWave + lane();
    const int i = e / N, j = e - i * N;
    if (e < T) A[i * L + j] = v[r];
  }
}
template <int LDN, int N, typename R, typename RG>
PKS_DEV void st_symm(const R* A, RG* g) {
  constexpr int L = ld<LDN>();
  for (int e = lane(); e < N * N; e += kWave) {
    const int i = e / N, j = e - i * N;
    if (j >= i) g[sym_index<N>(i, j)] = RG(A[i * L + j]);
  }
}
template <int N, typename RG, typename R>
PKS_DEV void ld_v(const RG* g, R* x) {
  for (int i = lane(); i < N; i += kWave) x[i] = R(g[i]);
}
template <int N, typename R, typename RG>
PKS_DEV void st_v(const R* x, RG* g) {
  for (int i = lane(); i < N; i += kWave) g[i] = RG(x[i]);
}

// ---------------------------------------------------------------------------
// Record layouts (words of one slot, contiguous in HBM).
// ---------------------------------------------------------------------------
template <int N, int P>
struct Layout {
  static constexpr int kS = sym_size<N>(), kSP = sym_size<P>();
  static constexpr int kTraj = N + kS;                     // mean, cov
  static constexpr int kTrans = N * N + N + kS;            // F, c, Q'
  static constexpr int kHlin = P * N + P + kSP + P;        // H, d, R', ytilde
  static constexpr int kFElem = N * N + 2 * N + 2 * kS;    // A, b, C, eta, J
  static constexpr int kSElem = N * N + N + kS;            // E, g, L
  static constexpr int kCarry = N + kS;                    // (b, C) or (g, L)
  static_assert(kSElem <= kFElem, "smoothing elements reuse the filtering element records");
};

// LDS work area of one wave: NM matrices of N x N (names per kernel), sized
// per kernel so that light kernels keep more waves resident.
template <int N, typename R, int NM>
struct Work {
  static constexpr int MW = mat_words<N>();
  static constexpr int kNM = NM;
  R m[NM][MW];
  R v[8][N];       // vectors
  int ok;
};

// --- restarts -------------------------------------------------------------
// A right operand with A = 0 (filtering) or E = 0 (smoothing) -- a track's
// prior or end element, or an aggregate that contains one -- yields its own
// (b, C) resp. (g, L) whatever the left operand holds.  The formulas give that
// for finite operands; when a failed left operand has turned the result into
// NaN (0 * NaN), the restart is taken as is, so a failed track never spills
// into the tracks after it.  Every lane reads the same LDS words, so the
// branch is uniform; finite results are unchanged bit for bit.
template <int N, typename R>
PKS_DEV bool all_zero(const R* A) {
  bool z = true;
  for (int e = lane(); e < N * N; e += kWave) z = z && A[(e / N) * ld<N>() + e % N] == R(0);
  return __all(z);
}

template <int N, typename R>
PKS_DEV void take_restart(const R* rA, const R* rb, const R* rC, R* lA, R* lb, R* lC) {
  constexpr int L = ld<N>();
  for (int e = lane(); e < N * N; e += kWave) {
    const int i = e / N, j = e - i * N;
    if (lA) lA[i * L + j] = R(0);
    lC[i * L + j] = rC[i * L + j];
  }
  for (int i = lane(); i < N; i += kWave) lb[i] = rb[i];
  wsync();
}

// --- the filtering operator (eq. 15), symmetric pivot-free form ------------
// l <- l (x) r with l = (lA, lb, lC, le, lJ), r = (rA, rb, C_j, re, rJ).  Same
// algebra as FilterOp::combine.  l's C holds its Cholesky factor and then M
// while the result is formed, S holds G, its factor and Y, rJ holds A_j M (rJ
// and S are destroyed), T is scratch.  C_j enters only the last step:
// getC(S) returns it as an LDS operand (it may read it into S, free by then).
template <int N, typename R, class GetC>
PKS_DEV void combine_f_impl(R* lA, R* lb, R* lC, R* le, R* lJ, const R* rA, const R* rb, const R* re, R* rJ, R* S,
                            R* T, R* v1, R* v2, int* ok, GetC getC) {
  mv<N, N, N, false>(rJ, lb, re, R(-1), v1);            // v = eta_j - J b_i
  chol<N, N>(lC, ok);                                   // U
  mm<N, N, N, N, false, false>(rJ, lC, (const R*)nullptr, R(1), T);      // J U
  mm<N, N, N, N, true, false>(lC, T, (const R*)nullptr, R(1), S);        // U^T J U
  for (int i = lane(); i < N; i += kWave) S[i * ld<N>() + i] += R(1);   // G
  wsync();
  chol<N, N>(S, ok);                                    // Lg
  copy<N, N, N, true>(lC, T);                           // U^T
  fwd<N, N, N>(S, T);                                   // W = Lg^-1 U^T
  mm<N, N, N, N, true, false>(T, T, (const R*)nullptr, R(1), lC);        // M = W^T W
  mm<N, N, N, N, false, false>(rJ, lA, (const R*)nullptr, R(1), S);      // Y = J A_i
  mm<N, N, N, N, false, false>(lC, S, (const R*)nullptr, R(1), T);       // Z = M Y
  mv<N, N, N, false>(lC, v1, (const R*)nullptr, R(1), v2);               // u = M v
  // J_ij = A_i^T Y - Y^T Z + J_i ; eta_ij = A_i^T v - Y^T u + eta_i
  mm<N, N, N, N, true, false>(lA, S, lJ, R(1), lJ);
  mm<N, N, N, N, true, false>(S, T, lJ, R(-1), lJ);
  mv<N, N, N, true>(lA, v1, le, R(1), le);
  mv<N, N, N, true>(S, v2, le, R(-1), le);
  symmetrize<N, N>(lJ);
  // b_ij = A_j (b_i + u) + b_j
  for (int i = lane(); i < N; i += kWave) v1[i] = lb[i] + v2[i];
  wsync();
  mv<N, N, N, false>(rA, v1, rb, R(1), lb);
  // C_ij = A_j M A_j^T + C_j
  mm<N, N, N, N, false, false>(rA, lC, (const R*)nullptr, R(1), rJ);     // A_j M
  const R* rC = getC(S);
  mm<N, N, N, N, false, true>(rJ, rA, rC, R(1), lC);
  symmetrize<N, N>(lC);
  // A_ij = A_j (A_i - Z)
  for (int e = lane(); e < N * N; e += kWave) {
    const int i = e / N, j = e - i * N;
    T[i * ld<N>() + j] = lA[i * ld<N>() + j] - T[i * ld<N>() + j];
  }
  wsync();
  mm<N, N, N, N, false, false>(rA, T, (const R*)nullptr, R(1), lA);
  if (!(lb[0] == lb[0]) && all_zero<N>(rA)) take_restart<N>(rA, rb, rC, lA, lb, lC);
}

// All operands in LDS; S and T scratch, rJ destroyed.  The routine-cycle probe
// times this form.
template <int N, typename R>
PKS_DEV void combine_f(R* lA, R* lb, R* lC, R* le, R* lJ, const R* rA, const R* rb, const R* rC, const R* re, R* rJ,
                       R* S, R* T, R* v1, R* v2, int* ok) {
  combine_f_impl<N, R>(lA, lb, lC, le, lJ, rA, rb, re, rJ, S, T, v1, v2, ok, [&](R*) { return rC; });
}

// The kernels' form: C_j stays in the right element's record in global memory
// (gC, symmetric packed, written before the call) and is read into rC, which
// serves as S until then; the right element takes two LDS matrices (rA, rJ)
// plus rC, and the call one scratch matrix T.
template <int N, typename R, typename RG>
PKS_DEV void combine_f_lean(R* lA, R* lb, R* lC, R* le, R* lJ, const R* rA, const R* rb, R* rC, const R* re,
                            R* rJ, const RG* gC, R* T, R* v1, R* v2, int* ok) {
  combine_f_impl<N, R>(lA, lb, lC, le, lJ, rA, rb, re, rJ, rC, T, v1, v2, ok, [&](R* buf) {
    ld_symm<N, N>(gC, buf);
    wsync();
    return static_cast<const R*>(buf);
  });
}

// Carry (b, C) (x) r: the filtered mean and covariance after element r.  The
// carry's covariance holds its Cholesky factor and then M while the result is
// formed, rJ holds G and its factor (rJ is destroyed), T is scratch.  The
// element's C enters only the last step: getC(rJ) returns it as an LDS
// operand (it may read it into rJ, free by then).
template <int N, typename R, class GetC>
PKS_DEV void apply_f_impl(R* cb, R* cC, const R* rA, const R* rb, const R* re, R* rJ, R* T, R* v1, R* v2, int* ok,
                          GetC getC) {
  mv<N, N, N, false>(rJ, cb, re, R(-1), v1);            // v = eta - J b, before rJ is reused
  chol<N, N>(cC, ok);                                   // U
  mm<N, N, N, N, false, false>(rJ, cC, (const R*)nullptr, R(1), T);      // J U
  mm<N, N, N, N, true, false>(cC, T, (const R*)nullptr, R(1), rJ);       // U^T J U
  for (int i = lane(); i < N; i += kWave) rJ[i * ld<N>() + i] += R(1);  // G
  wsync();
  chol<N, N>(rJ, ok);                                   // Lg
  copy<N, N, N, true>(cC, T);                           // U^T
  fwd<N, N, N>(rJ, T);                                  // W = Lg^-1 U^T
  mm<N, N, N, N, true, false>(T, T, (const R*)nullptr, R(1), cC);        // M = W^T W
  mv<N, N, N, false>(cC, v1, (const R*)nullptr, R(1), v2);               // u = M v
  for (int i = lane(); i < N; i += kWave) v1[i] = cb[i] + v2[i];
  wsync();
  mv<N, N, N, false>(rA, v1, rb, R(1), cb);
  mm<N, N, N, N, false, false>(rA, cC, (const R*)nullptr, R(1), T);      // A M
  const R* rC = getC(rJ);
  mm<N, N, N, N, false, true>(T, rA, rC, R(1), cC);     // A M A^T + C
  symmetrize<N, N>(cC);
  if (!(cb[0] == cb[0]) && all_zero<N>(rA)) take_restart<N>(rA, rb, rC, (R*)nullptr, cb, cC);
}

// All operands in LDS; one scratch matrix T, rJ destroyed.
template <int N, typename R>
PKS_DEV void apply_f(R* cb, R* cC, const R* rA, const R* rb, const R* rC, const R* re, R* rJ, R* T, R* v1, R* v2,
                     int* ok) {
  apply_f_impl<N, R>(cb, cC, rA, rb, re, rJ, T, v1, v2, ok, [&](R*) { return rC; });
}

// The element's C stays in its record in global memory (gC, symmetric packed)
// and is read into rJ's buffer for the last step: the element takes two LDS
// matrices (rA, rJ).
template <int N, typename R, typename RG>
PKS_DEV void apply_f_lean(R* cb, R* cC, const R* rA, const R* rb, const RG* gC, const R* re, R* rJ, R* T, R* v1,
                          R* v2, int* ok) {
  apply_f_impl<N, R>(cb, cC, rA, rb, re, rJ, T, v1, v2, ok, [&](R* buf) {
    ld_symm<N, N>(gC, buf);
    wsync();
    return static_cast<const R*>(buf);
  });
}

// --- the smoothing operator (eq. 19) ------------------------------------------
// l <- l (x) r in the paper's order (l earlier in time): (E_l E_r, E_l g_r + g_l, E_l L_r E_l^T + L_l).
// T1 and T2 are scratch and may be the same matrix.
template <int N, typename R>
PKS_DEV void combine_s(R* lE, R* lg, R* lL, const R* rE, const R* rg, const R* rL, R* T1, R* T2, R* v1) {
  // E_l = 0 (a track's end element or an aggregate holding one): the result
  // is l itself; l is updated in place, so the restart is taken up front.
  if (lE[0] == R(0) && all_zero<N>(lE)) return;
  mm<N, N, N, N, false, false>(lE, rL, (const R*)nullptr, R(1), T1);
  mm<N, N, N, N, false, true>(T1, lE, lL, R(1), lL);
  symmetrize<N, N>(lL);
  mv<N, N, N, false>(lE, rg, (const R*)nullptr, R(1), v1);
  mm<N, N, N, N, false, false>(lE, rE, (const R*)nullptr, R(1), T2);
  copy<N, N, N, false>(T2, lE);
  for (int i = lane(); i < N; i += kWave) lg[i] += v1[i];
  wsync();
}

// r (x) carry (g, L): the smoothed mean and covariance before the carry.
template <int N, typename R>
PKS_DEV void apply_s(const R* rE, const R* rg, const R* rL, R* cg, R* cL, R* T1, R* v1) {
  mm<N, N, N, N, false, false>(rE, cL, (const R*)nullptr, R(1), T1);
  mm<N, N, N, N, false, true>(T1, rE, rL, R(1), cL);
  symmetrize<N, N>(cL);
  mv<N, N, N, false>(rE, cg, rg, R(1), v1);
  vcopy<N>(v1, cg);
  if (!(cg[0] == cg[0] && cL[0] == cL[0]) && all_zero<N>(rE)) take_restart<N>(rE, rg, rL, (R*)nullptr, cg, cL);
}

// --- statistical linear regression (eq. 7-9) of g: R^N -> R^Q at (xbar, Pbar)
// with the symmetric sigma-point set of elements.hpp (slr): one sigma point
// per lane.  Inputs xbar (LDS vector) and Pbar (LDS matrix, destroyed: it
// becomes its Cholesky factor).  Outputs G (Q x N, LDS), off = zbar - G xbar,
// Lam (Q x Q), zc = g(xbar).  Zp, Zm, D: N x Q scratch; zbar: Q vector.  D may
// be Zp and G may be Zm (D is formed in place once Phi has read the images,
// G once D is done with them), so the regression fits in four matrices.
template <int N, int Q, bool kAngular, typename R, class Eval>
PKS_DEV void slr(int lin, SigmaRule rule, const R* xbar, R* Pbar, Eval eval, R* G, R* off, R* Lam, R* zc, R* Zp,
                 R* Zm, R* D, R* zbar, int* ok, bool factored = false) {
  constexpr int L = ld<N>();
  if (!factored) chol<N, N>(Pbar, ok);    // else Pbar already holds the factor
  R gamma, w0, wj;
  sigma_weights<N, R>(lin, rule, gamma, w0, wj);
  // all 2N + 1 points in one pass: lane 2N takes the centre
  static_assert(2 * N + 1 <= kWave, "one sigma point per lane");
  if (lane() <= 2 * N) {
    const bool centre = lane() == 2 * N;
    const int j = lane() < N ? lane() : (centre ? 0 : lane() - N);
    const R sg = lane() < N ? gamma : -gamma;
    R x[N], z[Q];
    PKS_UNROLL for (int i = 0; i < N; ++i) x[i] = centre ? xbar[i] : xbar[i] + sg * Pbar[i * L + j];
    eval(x, z);
    R* out = centre ? zc : (lane() < N ? Zp + j * L : Zm + j * L);
    PKS_UNROLL for (int q = 0; q < Q; ++q) out[q] = z[q];
  }
  wsync();
  if constexpr (kAngular) {   // each image on the branch of the centre's
    for (int e = lane(); e < 2 * N * Q; e += kWave) {
      const int jj = e / Q, q = e - jj * Q;
      R* v = (jj < N ? Zp + jj * L : Zm + (jj - N) * L) + q;
      *v = zc[q] + wrap_pi<R>(*v - zc[q]);
    }
    wsync();
  }
  for (int q = lane(); q < Q; q += kWave) {
    R s = R(0);
    for (int j = 0; j < N; ++j) s += Zp[j * L + q] + Zm[j * L + q];
    zbar[q] = w0 * zc[q] + wj * s;
  }
  wsync();
  // Lambda = Phi - D^T D, Phi = sum_j w_j (Z_j - zbar)(Z_j - zbar)^T
  for (int e = lane(); e < Q * Q; e += kWave) {
    const int a = e / Q, b = e - a * Q;
    if (b < a) continue;
    R s = R(0);
    for (int j = 0; j < N; ++j)
      s += (Zp[j * L + a] - zbar[a]) * (Zp[j * L + b] - zbar[b]) +
           (Zm[j * L + a] - zbar[a]) * (Zm[j * L + b] - zbar[b]);
    s = s * wj + w0 * (zc[a] - zbar[a]) * (zc[b] - zbar[b]);
    Lam[a * L + b] = s;
  }
  wsync();
  const R wg = wj * gamma;
  for (int e = lane(); e < N * Q; e += kWave) {
    const int j = e / Q, q = e - j * Q;
    D[j * L + q] = wg * (Zp[j * L + q] - Zm[j * L + q]);
  }
  wsync();
  for (int e = lane(); e < Q * Q; e += kWave) {
    const int a = e / Q, b = e - a * Q;
    if (b < a) continue;
    R s = Lam[a * L + b];
    for (int j = 0; j < N; ++j) s -= D[j * L + a] * D[j * L + b];
    Lam[a * L + b] = s;
    Lam[b * L + a] = s;
  }
  wsync();
  bwd<N, N, Q>(Pbar, D);                    // G^T = L^-T D
  copy<N, Q, N, true>(D, G);
  for (int q = lane(); q < Q; q += kWave) {
    R s = zbar[q];
    for (int i = 0; i < N; ++i) s -= G[q * L + i] * xbar[i];
    off[q] = s;
  }
  wsync();
}

// ---------------------------------------------------------------------------
// Kernel arguments.
// ---------------------------------------------------------------------------
struct DnArgs {
  int64_t S;
  int ntracks;
  int lin;
  SigmaRule rule;
  const unsigned char* flags;   // kSlotFirst / kSlotLast per slot
  const int* track;             // track of each slot
  const void* params;
  const void* Q;                // N x N full
  const void* Rm;               // P x P full
  const double* params64;       // the same three in FP64, for the linearisation
  const double* Q64;
  const double* Rm64;
  const void* m0;               // [track][N]
  const void* P0;               // [track][N][N] full
  const void* y;                // [slot][P] (slot 0 of a track unused)
  void* traj;                   // [slot][kTraj]
  void* trans;                  // [slot][kTrans]
  void* hlin;                   // [slot][kHlin]
  void* elem;                   // [slot][kFElem]; smoothing elements reuse it
  unsigned long long* delta_bits;
  double lm;                    // Levenberg-Marquardt damping lambda (0 = undamped)
};

// The same model in another precision (model templates are <N, P, real>).
template <class M, typename T>
struct WithReal;
template <template <int, int, typename> class Mt, int N, int P, typename R, typename T>
struct WithReal<Mt<N, P, R>, T> {
  using type = Mt<N, P, T>;
};

struct DnLevel {
  const void* in;    // aggregates of this level (count n)
  void* out;         // aggregates of the next level (count ceil(n / fan))
  void* carry_out;   // exclusive carries of this level's elements (count n)
  const void* carry_in;  // exclusive carries of the next level's chunks
  int64_t n;
  int fan;
};

template <class Model, typename R>
struct Dense {
  static constexpr int N = Model::N, P = Model::P;
  using Lay = Layout<N, P>;
  using W = Work<N, R, 9>;
  template <int NM>
  using WorkN = Work<N, R, NM>;

  // element a_s into (A, b, C, eta, J) in the given LDS buffers, with one
  // scratch matrix T: F and Q' are read into A's and C's buffers (A and C are
  // formed over them), S and H into rows 0..P-1 and P..2P-1 of J's buffer (J
  // is formed last), H Q' and H F into the same rows of T.  A work area of
  // nine matrices also takes the Levenberg-Marquardt damping (w.m[6..8]).
  template <class WT>
  static PKS_DEV void build_element(const DnArgs& a, int64_t s, WT& w, R* T, R* A, R* b, R* C, R* e, R* J) {
    static_assert(2 * P <= N, "S and H share one matrix buffer");
    constexpr int L = ld<N>();
    const unsigned fl = a.flags[s];
    if (fl & kSlotFirst) {
      const int tr = a.track[s];
      zero<N, N, N>(A);
      zero<N, N, N>(J);
      ld_v<N>(static_cast<const R*>(a.m0) + size_t(tr) * N, b);
      ld_full<N, N, N>(static_cast<const R*>(a.P0) + size_t(tr) * N * N, C);
      for (int i = lane(); i < N; i += kWave) e[i] = R(0);
      wsync();
      if constexpr (WT::kNM >= 9) {
        if (a.lm > 0.0) lm_damp(a, s, w, A, b, C, e, J);
      }
      return;
    }
    // transition out of slot s - 1, measurement at slot s
    const R* tr = static_cast<const R*>(a.trans) + size_t(s - 1) * Lay::kTrans;
    const R* hl = static_cast<const R*>(a.hlin) + size_t(s) * Lay::kHlin;
    R* F = A;
    R* Qp = C;
    R* Sx = J;          // P x P
    R* H = J + P * L;   // P x N
    R* c = w.v[4];
    R* d = w.v[5];
    R* yt = w.v[6];
    ld_full<N, N, N>(tr, F);
    ld_v<N>(tr + N * N, c);
    ld_symm<N, N>(tr + N * N + N, Qp);
    ld_full<N, P, N>(hl, H);
    ld_v<P>(hl + P * N, d);
    ld_symm<N, P>(hl + P * N + P, Sx);
    ld_v<P>(hl + P * N + P + Lay::kSP, yt);
    wsync();
    R* HQ = T;          // P x N
    R* HF = T + P * L;  // P x N
    mm<N, P, N, N, false, false>(H, Qp, (const R*)nullptr, R(1), HQ);
    mm<N, P, N, N, false, false>(H, F, (const R*)nullptr, R(1), HF);
    mm<N, P, N, P, false, true>(HQ, H, Sx, R(1), Sx);                      // S = H Q' H^T + R'
    chol<N, P>(Sx, &w.ok);
    mv<N, P, N, false>(H, c, yt, R(-1), yt);                                // w = y - H c - d
    for (int i = lane(); i < P; i += kWave) yt[i] -= d[i];
    wsync();
    fwd<N, P, N>(Sx, HQ);                                                   // Zs = Ls^-1 H Q'
    fwd<N, P, N>(Sx, HF);                                                   // Ys = Ls^-1 H F
    fwd_vec<N, P>(Sx, yt);                                                  // ws = Ls^-1 w
    mv<N, N, P, true>(HQ, yt, c, R(1), b);                                  // b = c + Zs^T ws
    mv<N, N, P, true>(HF, yt, (const R*)nullptr, R(1), e);                  // eta = Ys^T ws
    mm<N, N, P, N, true, false>(HQ, HF, F, R(-1), A);                       // A = F - Zs^T Ys
    mm<N, N, P, N, true, false>(HQ, HQ, Qp, R(-1), C);                      // C = Q' - Zs^T Zs
    mm<N, N, P, N, true, false>(HF, HF, (const R*)nullptr, R(1), J);       // J = Ys^T Ys
    symmetrize<N, N>(C);
    symmetrize<N, N>(J);
    if constexpr (WT::kNM >= 9) {
      if (a.lm > 0.0) lm_damp(a, s, w, A, b, C, e, J);
    }
  }

  // Levenberg-Marquardt damping of the element of slot s (Section 3, damped
  // Gauss-Newton extension): the previous iterate xbar_s is observed through
  // x_s with noise covariance I/lambda.  With G = I + lambda C = L L^T,
  // Z = L^-1 C, V = L^-1 A, v = L^-1 (xbar - b):
  //   A -= lambda Z^T V,  b += lambda Z^T v,  C -= lambda Z^T Z,
  //   J += lambda V^T V,  eta += lambda V^T v.
  // Scratch: w.m[6..8], w.v[4] (free once the element is built).
  template <class WT>
  static PKS_DEV void lm_damp(const DnArgs& a, int64_t s, WT& w, R* A, R* b, R* C, R* e, R* J) {
    constexpr int L = ld<N>();
    const R lam = R(a.lm);
    const R* xbar = static_cast<const R*>(a.traj) + size_t(s) * Lay::kTraj;
    R* G = w.m[6];
    R* Z = w.m[7];
    R* V = w.m[8];
    R* v = w.v[4];
    for (int t = lane(); t < N * N; t += kWave) {
      const int i = t / N, j = t - i * N;
      G[i * L + j] = lam * C[i * L + j] + (i == j ? R(1) : R(0));
      Z[i * L + j] = C[i * L + j];
      V[i * L + j] = A[i * L + j];
    }
    for (int i = lane(); i < N; i += kWave) v[i] = xbar[i] - b[i];
    wsync();
    chol<N, N>(G, &w.ok);
    fwd<N, N, N>(G, Z);
    fwd<N, N, N>(G, V);
    fwd_vec<N, N>(G, v);
    mv<N, N, N, true>(Z, v, b, lam, b);
    mv<N, N, N, true>(V, v, e, lam, e);
    mm<N, N, N, N, true, false>(Z, V, A, -lam, A);
    mm<N, N, N, N, true, false>(Z, Z, C, -lam, C);
    mm<N, N, N, N, true, false>(V, V, J, lam, J);
    symmetrize<N, N>(C);
    symmetrize<N, N>(J);
  }

  static PKS_DEV void store_felem(const R* A, const R* b, const R* C, const R* e, const R* J, R* g) {
    st_full<N, N, N>(A, g);
    st_v<N>(b, g + N * N);
    st_symm<N, N>(C, g + N * N + N);
    st_v<N>(e, g + N * N + N + Lay::kS);
    st_symm<N, N>(J, g + N * N + 2 * N + Lay::kS);
  }
  static PKS_DEV void load_felem(const R* g, R* A, R* b, R* C, R* e, R* J) {
    ld_full<N, N, N>(g, A);
    ld_v<N>(g + N * N, b);
    ld_symm<N, N>(g + N * N + N, C);
    ld_v<N>(g + N * N + N + Lay::kS, e);
    ld_symm<N, N>(g + N * N + 2 * N + Lay::kS, J);
    wsync();
  }
  static PKS_DEV void store_selem(const R* E, const R* g_, const R* Lm, R* g) {
    st_full<N, N, N>(E, g);
    st_v<N>(g_, g + N * N);
    st_symm<N, N>(Lm, g + N * N + N);
  }
  static PKS_DEV void load_selem(const R* g, R* E, R* g_, R* Lm) {
    ld_full<N, N, N>(g, E);
    ld_v<N>(g + N * N, g_);
    ld_symm<N, N>(g + N * N + N, Lm);
    wsync();
  }
  static PKS_DEV void store_carry(const R* x, const R* Pm, R* g) {
    st_v<N>(x, g);
    st_symm<N, N>(Pm, g + N);
  }
  static PKS_DEV void load_carry(const R* g, R* x, R* Pm) {
    ld_v<N>(g, x);
    ld_symm<N, N>(g + N, Pm);
    wsync();
  }
};

// ---------------------------------------------------------------------------
// Kernels.  Every workgroup is one wave (64 lanes).
// ---------------------------------------------------------------------------

// Linearisation of f (all but the last slot of a track) and h (all but the
// first) at the current trajectory; one slot per workgroup.
template <class Model, typename R>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3))) void k_dn_linearize(DnArgs a) {
  // The regression runs in FP64 whatever the records' type R: in FP32 its
  // sums of sigma-point images (z-bar - G x-bar, Phi - D^T D) would cost more
  // accuracy than the FP32 scan itself.
  using RC = double;
  using MC = typename WithReal<Model, RC>::type;
  using D = Dense<MC, RC>;
  constexpr int N = D::N, P = D::P;
  using Lay = typename D::Lay;
  __shared__ typename D::template WorkN<4> w;   // Pbar's factor; images and D; images and G; Lambda
  const int64_t s = blockIdx.x;
  if (s >= a.S) return;
  if (lane() == 0) w.ok = 1;
  const MC md{a.params64};
  const unsigned fl = a.flags[s];
  const R* tj = static_cast<const R*>(a.traj) + size_t(s) * Lay::kTraj;
  RC* xbar = w.v[0];
  ld_v<N>(tj, xbar);
  wsync();
  bool factored = false;   // w.m[0] holds the Cholesky factor of Pbar, shared by f and h
  if (!(fl & kSlotLast)) {
    ld_symm<N, N>(tj + N, w.m[0]);
    wsync();
    RC* G = w.m[2];
    RC* Lam = w.m[3];
    slr<N, N, false, RC>(a.lin, a.rule, xbar, w.m[0], [&](const RC(&x)[N], RC(&z)[N]) { md.f(x, z); }, G, w.v[1],
                         Lam, w.v[2], w.m[1], w.m[2], w.m[1], w.v[3], &w.ok);
    factored = true;
    R* out = static_cast<R*>(a.trans) + size_t(s) * Lay::kTrans;
    add_full<N, N, N>(a.Q64, Lam);
    wsync();
    st_full<N, N, N>(G, out);
    st_v<N>(w.v[1], out + N * N);
    st_symm<N, N>(Lam, out + N * N + N);
    wsync();                      // the stores have read LDS before it is reused
  }
  if (!(fl & kSlotFirst)) {
    if (!factored) {
      ld_symm<N, N>(tj + N, w.m[0]);
      wsync();
    }
    RC* H = w.m[2];
    RC* Om = w.m[3];
    RC* hc = w.v[2];
    slr<N, P, MC::kAngular, RC>(a.lin, a.rule, xbar, w.m[0], [&](const RC(&x)[N], RC(&z)[P]) { md.h(x, z); }, H,
                                w.v[1], Om, hc, w.m[1], w.m[2], w.m[1], w.v[3], &w.ok, factored);
    R* out = static_cast<R*>(a.hlin) + size_t(s) * Lay::kHlin;
    const R* y = static_cast<const R*>(a.y) + size_t(s) * P;
    add_full<N, P, P>(a.Rm64, Om);
    for (int i = lane(); i < P; i += kWave)
      out[P * N + P + Lay::kSP + i] = R(MC::kAngular ? hc[i] + wrap_pi<RC>(RC(y[i]) - hc[i]) : RC(y[i]));
    wsync();
    st_full<N, P, N>(H, out);
    st_v<P>(w.v[1], out + P * N);
    st_symm<N, P>(Om, out + P * N + P);
  }
}

// Level 0 of the filtering scan: build the elements of `fan` consecutive
// slots, store them, and fold them into the chunk aggregate.  The aggregate,
// the element being folded in and one scratch matrix take seven matrices
// (24.8 KB in FP64: six waves per CU); the damped form (kDamp, lambda > 0)
// has two more for the damping.
template <class Model, typename R, bool kDamp>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 2))) void k_dn_forward_up(DnArgs a, int fan, void* agg_out) {
  using D = Dense<Model, R>;
  constexpr int N = D::N;
  using Lay = typename D::Lay;
  __shared__ typename D::template WorkN<kDamp ? 9 : 7> w;
  if (lane() == 0) w.ok = 1;
  const int64_t s0 = int64_t(blockIdx.x) * fan;
  const int64_t s1 = min(s0 + fan, a.S);
  R *lA = w.m[0], *lC = w.m[1], *lJ = w.m[2], *rA = w.m[3], *rJ = w.m[4], *rC = w.m[5], *T = w.m[6];
  R *lb = w.v[0], *le = w.v[1], *rb = w.v[2], *re = w.v[3];
  for (int64_t s = s0; s < s1; ++s) {
    R* A = s == s0 ? lA : rA;
    R* C = s == s0 ? lC : rC;
    R* J = s == s0 ? lJ : rJ;
    R* b = s == s0 ? lb : rb;
    R* e = s == s0 ? le : re;
    R* rec = static_cast<R*>(a.elem) + size_t(s) * Lay::kFElem;
    D::build_element(a, s, w, T, A, b, C, e, J);
    D::store_felem(A, b, C, e, J, rec);
    if (s > s0)
      combine_f_lean<N, R>(lA, lb, lC, le, lJ, rA, rb, rC, re, rJ, rec + N * N + N, T, w.v[4], w.v[5], &w.ok);
  }
  D::store_felem(lA, lb, lC, le, lJ, static_cast<R*>(agg_out) + size_t(blockIdx.x) * Lay::kFElem);
}

// Up-sweep of a scan level: fold `fan` consecutive aggregates.  FILT selects
// the operator (filtering: records of kFElem words; smoothing: kSElem).
template <class Model, bool FILT, typename R>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_dn_scan_up(DnArgs a, DnLevel lv) {
  using D = Dense<Model, R>;
  constexpr int N = D::N;
  using Lay = typename D::Lay;
  constexpr int RW = FILT ? Lay::kFElem : Lay::kSElem;
  __shared__ typename D::template WorkN<FILT ? 7 : 6> w;
  if (lane() == 0) w.ok = 1;
  const int64_t i0 = int64_t(blockIdx.x) * lv.fan;
  const int64_t i1 = min(i0 + lv.fan, lv.n);
  const R* in = static_cast<const R*>(lv.in);
  R* out = static_cast<R*>(lv.out) + size_t(blockIdx.x) * RW;
  if (FILT) {
    D::load_felem(in + size_t(i0) * RW, w.m[0], w.v[0], w.m[1], w.v[1], w.m[2]);
    for (int64_t i = i0 + 1; i < i1; ++i) {
      // the right operand's C stays in its record until the combine's last step
      const R* g = in + size_t(i) * RW;
      ld_full<N, N, N>(g, w.m[3]);
      ld_v<N>(g + N * N, w.v[2]);
      ld_v<N>(g + N * N + N + Lay::kS, w.v[3]);
      ld_symm<N, N>(g + N * N + 2 * N + Lay::kS, w.m[5]);
      wsync();
      combine_f_lean<N, R>(w.m[0], w.v[0], w.m[1], w.v[1], w.m[2], w.m[3], w.v[2], w.m[4], w.v[3], w.m[5],
                           g + N * N + N, w.m[6], w.v[4], w.v[5], &w.ok);
    }
    D::store_felem(w.m[0], w.v[0], w.m[1], w.v[1], w.m[2], out);
  } else {
    D::load_selem(in + size_t(i0) * RW, w.m[0], w.v[0], w.m[1]);
    for (int64_t i = i0 + 1; i < i1; ++i) {
      D::load_selem(in + size_t(i) * RW, w.m[2], w.v[1], w.m[3]);
      combine_s<N, R>(w.m[0], w.v[0], w.m[1], w.m[2], w.v[1], w.m[3], w.m[4], w.m[5], w.v[2]);
    }
    D::store_selem(w.m[0], w.v[0], w.m[1], out);
  }
}

// Down-sweep of a scan level: exclusive carries of the `fan` aggregates of one
// chunk from the chunk's own exclusive carry.  Filtering runs forward (the
// first element overall has no carry: it starts at a prior element);
// smoothing runs backward (the last element overall has none: it ends at a
// last slot).
template <class Model, bool FILT, typename R>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_dn_scan_down(DnArgs a, DnLevel lv) {
  using D = Dense<Model, R>;
  constexpr int N = D::N;
  using Lay = typename D::Lay;
  constexpr int RW = FILT ? Lay::kFElem : Lay::kSElem;
  __shared__ typename D::template WorkN<5> w;
  if (lane() == 0) w.ok = 1;
  const int64_t c = blockIdx.x;
  const int64_t i0 = c * lv.fan;
  const int64_t i1 = min(i0 + lv.fan, lv.n);
  const int64_t nchunks = (lv.n + lv.fan - 1) / lv.fan;
  const R* in = static_cast<const R*>(lv.in);
  R* cout = static_cast<R*>(lv.carry_out);
  R *cx = w.v[6], *cP = w.m[4];
  R *rA = w.m[0], *rC = w.m[1], *rJ = w.m[2], *rb = w.v[0], *re = w.v[1];
  bool have = FILT ? c > 0 : c < nchunks - 1;
  if (have) D::load_carry(static_cast<const R*>(lv.carry_in) + size_t(c) * Lay::kCarry, cx, cP);
  for (int64_t k = 0; k < i1 - i0; ++k) {
    const int64_t i = FILT ? i0 + k : i1 - 1 - k;
    if (have) {
      D::store_carry(cx, cP, cout + size_t(i) * Lay::kCarry);
      wsync();
    }
    if (k + 1 == i1 - i0) break;   // the carry past the chunk's last aggregate is not needed
    if (FILT) {
      D::load_felem(in + size_t(i) * RW, rA, rb, rC, re, rJ);
      if (have) {
        apply_f<N, R>(cx, cP, rA, rb, rC, re, rJ, w.m[3], w.v[2], w.v[3], &w.ok);
      } else {
        vcopy<N>(rb, cx);
        copy<N, N, N, false>(rC, cP);
      }
    } else {
      D::load_selem(in + size_t(i) * RW, rA, rb, rC);
      if (have) {
        apply_s<N, R>(rA, rb, rC, cx, cP, w.m[3], w.v[2]);
      } else {
        vcopy<N>(rb, cx);
        copy<N, N, N, false>(rC, cP);
      }
    }
    have = true;
  }
}

// Level 0 down-sweep of the filtering scan and level 0 up-sweep of the
// smoothing scan: filtered x*, P* of every slot of the chunk, its smoothing
// element (eq. 17-18, stored over the filtering element) and the chunk's
// smoothing aggregate.
template <class Model, typename R>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 2))) void k_dn_forward_down_backward_up(DnArgs a, int fan, const void* carry_in,
                                                                       void* sagg_out) {
  using D = Dense<Model, R>;
  constexpr int N = D::N;
  using Lay = typename D::Lay;
  constexpr int L = ld<N>();
  __shared__ typename D::template WorkN<6> w;
  if (lane() == 0) w.ok = 1;
  const int64_t c = blockIdx.x;
  const int64_t s0 = c * fan;
  const int64_t s1 = min(s0 + fan, a.S);
  R *cx = w.v[6], *cP = w.m[3];                       // filtered mean / covariance (carry)
  R *rA = w.m[0], *rJ = w.m[1], *T = w.m[2], *rb = w.v[0], *re = w.v[1];
  R *sE = w.m[4], *sL = w.m[5], *sg = w.v[7];          // smoothing aggregate
  bool have = c > 0;
  if (have) D::load_carry(static_cast<const R*>(carry_in) + size_t(c) * Lay::kCarry, cx, cP);
  for (int64_t s = s0; s < s1; ++s) {
    R* rec = static_cast<R*>(a.elem) + size_t(s) * Lay::kFElem;
    const R* recC = rec + N * N + N;                   // the element's C stays in the record
    ld_full<N, N, N>(rec, rA);
    ld_v<N>(rec + N * N, rb);
    ld_v<N>(rec + N * N + N + Lay::kS, re);
    ld_symm<N, N>(rec + N * N + 2 * N + Lay::kS, rJ);
    wsync();
    if (have) {
      apply_f_lean<N, R>(cx, cP, rA, rb, recC, re, rJ, T, w.v[2], w.v[3], &w.ok);
    } else {
      vcopy<N>(rb, cx);
      ld_symm<N, N>(recC, cP);
      wsync();
    }
    have = true;
    // smoothing element of slot s into (eE, eg, eL) = (m[0], rb, m[1]): the
    // filtering element is spent
    R *eE = w.m[0], *eg = rb, *eL = w.m[1];
    if (a.flags[s] & kSlotLast) {
      zero<N, N, N>(eE);
      vcopy<N>(cx, eg);
      copy<N, N, N, false>(cP, eL);
    } else {
      const R* tr = static_cast<const R*>(a.trans) + size_t(s) * Lay::kTrans;
      R *F = w.m[1], *FP = w.m[2], *Pp = w.m[0], *V = w.m[2];
      R *r = w.v[2], *t = w.v[3];
      ld_full<N, N, N>(tr, F);
      ld_symm<N, N>(tr + N * N + N, Pp);
      ld_v<N>(tr + N * N, r);
      wsync();
      mm<N, N, N, N, false, false>(F, cP, (const R*)nullptr, R(1), FP);   // F P*
      mm<N, N, N, N, false, true>(FP, F, Pp, R(1), Pp);                  // F P* F^T + Q'
      symmetrize<N, N>(Pp);
      mv<N, N, N, false>(F, cx, r, R(1), t);                              // F x* + c
      chol<N, N>(Pp, &w.ok);
      fwd<N, N, N>(Pp, V);                                                // V = Lp^-1 F P*
      fwd_vec<N, N>(Pp, t);
      mm<N, N, N, N, true, false>(V, V, cP, R(-1), eL);                   // L_s = P* - V^T V
      symmetrize<N, N>(eL);
      mv<N, N, N, true>(V, t, cx, R(-1), eg);                             // g = x* - V^T Lp^-1 (F x* + c)
      bwd<N, N, N>(Pp, V);                                                // E^T = Lp^-T V
      copy<N, N, N, true>(V, eE);
    }
    D::store_selem(eE, eg, eL, rec);
    if (s == s0) {
      copy<N, N, N, false>(eE, sE);
      copy<N, N, N, false>(eL, sL);
      vcopy<N>(eg, sg);
    } else {
      combine_s<N, R>(sE, sg, sL, eE, eg, eL, T, T, w.v[2]);
    }
  }
  (void)L;
  D::store_selem(sE, sg, sL, static_cast<R*>(sagg_out) + size_t(c) * Lay::kSElem);
}

// Level 0 down-sweep of the smoothing scan: the new trajectory (eq. 19) and the
// per-track largest change of the means.
template <class Model, typename R>
__global__ __launch_bounds__(kWave) void k_dn_backward_down(DnArgs a, int fan, const void* carry_in) {
  using D = Dense<Model, R>;
  constexpr int N = D::N;
  using Lay = typename D::Lay;
  __shared__ typename D::template WorkN<4> w;
  __shared__ R dmax[kWave];
  if (lane() == 0) w.ok = 1;
  const int64_t c = blockIdx.x;
  const int64_t s0 = c * fan;
  const int64_t s1 = min(s0 + fan, a.S);
  const int64_t nchunks = (a.S + fan - 1) / fan;
  R *cx = w.v[6], *cP = w.m[3];
  R *rE = w.m[0], *rL = w.m[1], *rg = w.v[0];
  bool have = c < nchunks - 1;
  if (have) D::load_carry(static_cast<const R*>(carry_in) + size_t(c) * Lay::kCarry, cx, cP);
  // running largest change of the current track segment of this chunk (lane 0);
  // published once per segment, and only when it exceeds the stored value
  int seg_track = -1;
  unsigned long long seg_bits = 0ull, all_bits = 0ull;
  auto publish = [&](unsigned long long* p, unsigned long long v) {
    if (v > *static_cast<volatile unsigned long long*>(p)) atomicMax(p, v);
  };
  for (int64_t k = 0; k < s1 - s0; ++k) {
    const int64_t s = s1 - 1 - k;
    D::load_selem(static_cast<const R*>(a.elem) + size_t(s) * Lay::kFElem, rE, rg, rL);
    if (have) {
      apply_s<N, R>(rE, rg, rL, cx, cP, w.m[2], w.v[2]);
    } else {
      vcopy<N>(rg, cx);
      copy<N, N, N, false>(rL, cP);
    }
    have = true;
    R* tj = static_cast<R*>(a.traj) + size_t(s) * Lay::kTraj;
    R m = R(0);
    bool nan = false;
    if (lane() < N) {
      const R d = fabs(cx[lane()] - tj[lane()]);
      nan = !(d == d);
      m = d;
    }
    dmax[lane()] = nan ? R(-1) : m;
    wsync();
    D::store_carry(cx, cP, tj);
    if (lane() == 0) {
      R mx = R(0);
      bool bad = false;
      for (int i = 0; i < N; ++i) {
        bad = bad || dmax[i] < R(0);
        mx = dmax[i] > mx ? dmax[i] : mx;
      }
      const unsigned long long bits = order_bits(bad ? __builtin_nan("") : double(mx));
      const int tr = a.track[s];
      if (tr != seg_track) {
        if (seg_track >= 0) publish(&a.delta_bits[seg_track], seg_bits);
        seg_track = tr;
        seg_bits = 0ull;
      }
      seg_bits = bits > seg_bits ? bits : seg_bits;
      all_bits = bits > all_bits ? bits : all_bits;
    }
    wsync();
  }
  if (lane() == 0 && seg_track >= 0) {
    publish(&a.delta_bits[seg_track], seg_bits);
    publish(&a.delta_bits[a.ntracks], all_bits);
  }
}

// Filtering pass only (Section 2: the filter is the prefix of the filtering
// elements): level 0 down-sweep that stores the filtered x*, P* of every slot
// of the chunk as a trajectory-layout record [slot][kTraj].
template <class Model, typename R>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_dn_forward_down_filter(DnArgs a, int fan, const void* carry_in,
                                                                  void* filt) {
  using D = Dense<Model, R>;
  constexpr int N = D::N;
  using Lay = typename D::Lay;
  __shared__ typename D::template WorkN<5> w;
  if (lane() == 0) w.ok = 1;
  const int64_t c = blockIdx.x;
  const int64_t s0 = c * fan;
  const int64_t s1 = min(s0 + fan, a.S);
  R *cx = w.v[6], *cP = w.m[4];
  R *rA = w.m[0], *rC = w.m[1], *rJ = w.m[2], *rb = w.v[0], *re = w.v[1];
  bool have = c > 0;
  if (have) D::load_carry(static_cast<const R*>(carry_in) + size_t(c) * Lay::kCarry, cx, cP);
  for (int64_t s = s0; s < s1; ++s) {
    D::load_felem(static_cast<const R*>(a.elem) + size_t(s) * Lay::kFElem, rA, rb, rC, re, rJ);
    if (have) {
      apply_f<N, R>(cx, cP, rA, rb, rC, re, rJ, w.m[3], w.v[2], w.v[3], &w.ok);
    } else {
      vcopy<N>(rb, cx);
      copy<N, N, N, false>(rC, cP);
    }
    have = true;
    D::store_carry(cx, cP, static_cast<R*>(filt) + size_t(s) * Lay::kTraj);
  }
}

// Log predictive density of slot s, log N(ytil_s; H_s m-_s + d_s, S_s) with
// m-_s = F x*_{s-1} + c, P-_s = F P*_{s-1} F^T + Q', S_s = H P-_s H^T + R'
// (the normalising constants that eq. 14 leaves out; summed over a track they
// give log p(y_{1:T}) of the linearised model), from the filtered moments of
// slot s-1; 0 at the first slot of a track.  One slot per workgroup.
template <class Model, typename R>
__global__ __launch_bounds__(kWave) void k_dn_loglik(DnArgs a, const void* filt, double* slot_ll) {
  using D = Dense<Model, R>;
  constexpr int N = D::N, P = D::P;
  using Lay = typename D::Lay;
  constexpr int L = ld<N>();
  __shared__ typename D::template WorkN<6> w;
  const int64_t s = blockIdx.x;
  if (a.flags[s] & kSlotFirst) {
    if (lane() == 0) slot_ll[s] = 0.0;
    return;
  }
  if (lane() == 0) w.ok = 1;
  const R* tr = static_cast<const R*>(a.trans) + size_t(s - 1) * Lay::kTrans;
  const R* hl = static_cast<const R*>(a.hlin) + size_t(s) * Lay::kHlin;
  const R* fp = static_cast<const R*>(filt) + size_t(s - 1) * Lay::kTraj;
  R *F = w.m[0], *Pf = w.m[1], *Pp = w.m[2], *HP = w.m[3], *H = w.m[4], *Sx = w.m[5];
  R *xf = w.v[0], *mp = w.v[1], *c = w.v[2], *d = w.v[3], *yt = w.v[4];
  ld_full<N, N, N>(tr, F);
  ld_v<N>(tr + N * N, c);
  ld_symm<N, N>(tr + N * N + N, Pp);
  ld_v<N>(fp, xf);
  ld_symm<N, N>(fp + N, Pf);
  ld_full<N, P, N>(hl, H);
  ld_v<P>(hl + P * N, d);
  ld_symm<N, P>(hl + P * N + P, Sx);
  ld_v<P>(hl + P * N + P + Lay::kSP, yt);
  wsync();
  mm<N, N, N, N, false, false>(F, Pf, (const R*)nullptr, R(1), HP);      // F P*
  mm<N, N, N, N, false, true>(HP, F, Pp, R(1), Pp);                      // P- = F P* F^T + Q'
  mv<N, N, N, false>(F, xf, c, R(1), mp);                                // m- = F x* + c
  mm<N, P, N, N, false, false>(H, Pp, (const R*)nullptr, R(1), HP);      // H P-
  mm<N, P, N, P, false, true>(HP, H, Sx, R(1), Sx);                      // S = H P- H^T + R'
  symmetrize<N, P>(Sx);
  chol<N, P>(Sx, &w.ok);
  mv<N, P, N, false>(H, mp, yt, R(-1), yt);                              // ytil - H m-
  for (int i = lane(); i < P; i += kWave) yt[i] -= d[i];
  wsync();
  fwd_vec<N, P>(Sx, yt);
  if (lane() == 0) {
    double quad = 0.0, logdet = 0.0;
    for (int i = 0; i < P; ++i) {
      quad += double(yt[i]) * double(yt[i]);
      logdet += 2.0 * log(double(Sx[i * L + i]));
    }
    constexpr double kLog2Pi = 1.8378770664093454836;
    slot_ll[s] = w.ok ? -0.5 * (P * kLog2Pi + logdet + quad) : __builtin_nan("");
  }
}

// Prior broadcast of the initial trajectory: (m0, P0) of the slot's track.
template <int N, typename R>
__global__ void k_dn_prior(int64_t S, const int* track, const R* m0, const R* P0, R* traj) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  constexpr int TW = N + sym_size<N>();
  if (e >= S * TW) return;
  const int64_t s = e / TW;
  const int k = int(e - s * TW);
  const int tr = track[s];
  if (k < N) {
    traj[e] = m0[size_t(tr) * N + k];
  } else {
    int i = 0, rem = k - N;
    while (rem >= N - i) {
      rem -= N - i;
      ++i;
    }
    traj[e] = P0[(size_t(tr) * N + i) * N + i + rem];
  }
}

// Caller layout <-> slot records: mean [S][N], cov [S][N][N].
template <int N, typename R>
__global__ void k_dn_unpack(int64_t S, const R* traj, R* mean, R* cov) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= S * N * N) return;
  const int64_t s = e / (N * N);
  const int r = int(e - s * N * N), i = r / N, j = r - i * N;
  const R* t = traj + size_t(s) * (N + sym_size<N>());
  if (cov) cov[e] = t[N + sym_index<N>(i, j)];
  if (mean && j == 0) mean[s * N + i] = t[i];
}

template <int N, typename R>
__global__ void k_dn_pack(int64_t S, const R* mean, const R* cov, SymConst<N, R> cc, int use_const, const int* track,
                          const R* P0, R* traj) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  constexpr int TW = N + sym_size<N>();
  if (e >= S * TW) return;
  const int64_t s = e / TW;
  const int k = int(e - s * TW);
  if (k < N) {
    traj[e] = mean[s * N + k];
    return;
  }
  int i = 0, rem = k - N;
  while (rem >= N - i) {
    rem -= N - i;
    ++i;
  }
  const int j = i + rem;
  if (cov)
    traj[e] = R(0.5) * (cov[(s * N + i) * N + j] + cov[(s * N + j) * N + i]);
  else if (use_const)
    traj[e] = cc.v[k - N];
  else
    traj[e] = P0[(size_t(track[s]) * N + i) * N + j];
}

}  // namespace dn
}  // namespace pks
