// MAP objective of a trajectory and the per-track bookkeeping of
// Levenberg-Marquardt iterations with a damping schedule.
//
// Section 3: the iterated extended smoother is Gauss-Newton on
//   J(x_{0:T}) = 1/2 |x_0 - m0|^2_{P0^-1}
//              + sum_k 1/2 |x_k - f(x_{k-1})|^2_{Q^-1} + 1/2 |y_k - h(x_k)|^2_{R^-1},
// and its Levenberg-Marquardt extension keeps a damped step only when J does
// not rise.  Bearing residuals are taken modulo 2 pi in [-pi, pi), the same
// unwrapping the linearisation applies.  The weights come in as whitening
// matrices W (lower triangular, W A W^T = I for A = Q, R, P0), so each term is
// 1/2 |W r|^2.
//
// Slot s of the batch contributes its prior term (first slot of a track) or
// its transition and measurement terms; the per-track sums then run in a
// fixed order (chunks of a track in parallel, chunk totals in sequence), so
// the objective is deterministic.
#pragma once

#include "slot_kernels.hpp"

namespace pks {

struct CostArgs {
  int64_t S;
  size_t stride;
  int ntracks;
  const unsigned char* flags;
  const int* track;
  const void* params;
  const void* m0;       // [N][ntracks]
  const void* yslot;    // [P][stride]
  const void* traj;     // [N + s(N)][stride], means in the first N rows
  const void* wq;       // N x N row-major lower triangular
  const void* wr;       // P x P
  const void* wp0;      // [ntracks][N][N]
  double* slot_cost;    // [S], slot order
  SlotMap map;          // slot -> column of the per-slot arrays
  // Record layouts: entry e of slot s's mean is traj[e * stride + col * traj_scale]
  // (col = map.col(s)), of its measurement yslot[e * stride + col * y_scale],
  // entry e of track t's m0 is m0[e * m0_stride + t * m0_scale].  Structure of
  // arrays: scales 1, m0_stride = ntracks; slot-major records: stride 1.
  int64_t traj_scale, y_scale;
  size_t m0_stride;
  int64_t m0_scale;
};

template <int N, typename R>
PKS_DEV R half_sq_whitened(const R* W, const R (&r)[N]) {
  R s = R(0);
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    R z = R(0);
    PKS_UNROLL for (int j = 0; j <= i; ++j) z += W[i * N + j] * r[j];
    s += z * z;
  }
  return R(0.5) * s;
}

// One lane per column of the per-slot arrays, launched over the padded
// column range; the result goes to slot order.
template <class Model, typename R>
__global__ __launch_bounds__(kSlotBlock) void k_objective_slots(CostArgs a) {
  constexpr int N = Model::N, P = Model::P;
  const int64_t cs = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  const int64_t s = a.map.slot(cs);
  if (s >= a.S) return;
  const R* traj = static_cast<const R*>(a.traj);
  R x[N], r[N];
  ld_vec<N>(traj, a.stride, cs * a.traj_scale, x);
  R c;
  if (a.flags[s] & kSlotFirst) {
    const int tr = a.track[s];
    R m0[N];
    ld_vec<N>(static_cast<const R*>(a.m0), a.m0_stride, tr * a.m0_scale, m0);
    PKS_UNROLL for (int i = 0; i < N; ++i) r[i] = x[i] - m0[i];
    c = half_sq_whitened<N, R>(static_cast<const R*>(a.wp0) + size_t(tr) * N * N, r);
  } else {
    const Model md{static_cast<const R*>(a.params)};
    R xp[N], fx[N], hx[P], y[P], e[P];
    ld_vec<N>(traj, a.stride, a.map.col(s - 1) * a.traj_scale, xp);
    md.f(xp, fx);
    PKS_UNROLL for (int i = 0; i < N; ++i) r[i] = x[i] - fx[i];
    c = half_sq_whitened<N, R>(static_cast<const R*>(a.wq), r);
    md.h(x, hx);
    ld_vec<P>(static_cast<const R*>(a.yslot), a.stride, cs * a.y_scale, y);
    PKS_UNROLL for (int i = 0; i < P; ++i) e[i] = Model::kAngular ? wrap_pi<R>(y[i] - hx[i]) : y[i] - hx[i];
    c += half_sq_whitened<P, R>(static_cast<const R*>(a.wr), e);
  }
  a.slot_cost[s] = double(c);
}

constexpr int kTrackSumB = 256;
constexpr int64_t kSumChunk = 4096;   // slots per partial sum

// Per-track sums in a fixed order, in two steps so that a long track is
// spread over many workgroups: workgroup (t, c) sums chunk c of track t
// (kSumChunk slots) into partial[c * ntracks + t] (0 past the track's end),
// then one lane per track adds its chunks in order.
static __global__ __launch_bounds__(kTrackSumB) void k_track_partials(const double* v, const int64_t* slot_off,
                                                                      int ntracks, double* partial) {
  __shared__ double red[kTrackSumB];
  const int t = blockIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t end = slot_off[t + 1];
  const int64_t lo = slot_off[t] + c * kSumChunk;
  const int64_t hi = lo + kSumChunk < end ? lo + kSumChunk : end;
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kTrackSumB) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kTrackSumB / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[c * ntracks + t] = red[0];
}

static __global__ __launch_bounds__(kTrackSumB) void k_track_totals(const double* partial, int ntracks, int nchunks,
                                                                    double* out) {
  const int t = int(blockIdx.x) * kTrackSumB + int(threadIdx.x);
  if (t >= ntracks) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += partial[size_t(c) * ntracks + t];
  out[t] = s;
}

// ---------------------------------------------------------------------------
// Log marginal likelihood of one linearised pass (Section 2: the filtering
// prefix carries p(y_{1:k}) with its normalising constants).  By the chain
// rule log p(y_{1:T}) = sum_k log p(y_k | y_{1:k-1}); each term is the
// Gaussian predictive density of the surrogate model at slot k,
//   N(ytil_k; H_k m-_k + d_k, S_k),  m-_k = F x*_{k-1} + c,
//   S_k = H_k (F P*_{k-1} F^T + Q') H_k^T + R'_k,
// from the filtered moments of slot k-1.  The first slot of a track has no
// measurement and contributes 0.
// ---------------------------------------------------------------------------
struct LoglikArgs {
  int64_t S;
  size_t stride;
  const unsigned char* flags;
  const void* params;
  const void* Q;        // N x N
  const void* R;        // P x P
  const void* yslot;    // [P][stride]
  const void* traj;     // linearisation points (Taylor rows are rebuilt from them)
  const void* trans;    // transition rows (TransLayout) of each slot; null: Taylor, rebuilt
  const void* lin;      // optional LinLayout rows with the stored measurement linearisation
  const void* filt;     // [N + s(N)][stride] filtered moments
  SigmaRule rule;
  double* slot_ll;      // [S], slot order
  SlotMap map;          // slot -> column of the per-slot arrays
};

template <class Model, typename R>
__global__ __launch_bounds__(kSlotBlock) void k_loglik_slots(LoglikArgs a) {
  constexpr int N = Model::N, P = Model::P;
  using TL = TransLayout<N>;
  using LL = LinLayout<N, P>;
  const int64_t s = a.map.slot(int64_t(blockIdx.x) * kSlotBlock + threadIdx.x);
  if (s >= a.S) return;
  if (a.flags[s] & kSlotFirst) {
    a.slot_ll[s] = 0.0;
    return;
  }
  const size_t st = a.stride;
  const int64_t cp = a.map.col(s - 1), cs = a.map.col(s);
  R F[N][N], c[N], Qp[N][N], H[P][N], d[P], Rp[P][P], yt[P];
  if (a.trans) {
    const R* tr = static_cast<const R*>(a.trans);
    ld_mat<N, N>(tr + TL::kF * st, st, cp, F);
    ld_vec<N>(tr + TL::kc * st, st, cp, c);
    ld_sym<N>(tr + TL::kQ * st, st, cp, Qp);
  } else {
    // Taylor transition at the linearisation point of slot k-1
    const Model md{static_cast<const R*>(a.params)};
    R xp[N], Pz[N][N], Qm[N][N];
    ld_vec<N>(static_cast<const R*>(a.traj), st, cp, xp);
    set_zero<N>(Pz);
    const R* Qg = static_cast<const R*>(a.Q);
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Qm[i][j] = Qg[i * N + j];
    linearize_f<Model, R>(md, kTaylor, a.rule, Qm, xp, Pz, F, c, Qp);
  }
  if (a.lin) {
    const R* lin = static_cast<const R*>(a.lin);
    ld_mat<P, N>(lin + LL::kH * st, st, cs, H);
    ld_vec<P>(lin + LL::kd * st, st, cs, d);
    ld_sym<P>(lin + LL::kR * st, st, cs, Rp);
    ld_vec<P>(lin + LL::ky * st, st, cs, yt);
  } else {
    const Model md{static_cast<const R*>(a.params)};
    R x[N], Px[N][N], Rm[P][P], y[P];
    ld_vec<N>(static_cast<const R*>(a.traj), st, cs, x);
    set_zero<N>(Px);
    const R* Rg = static_cast<const R*>(a.R);
    PKS_UNROLL for (int i = 0; i < P; ++i) PKS_UNROLL for (int j = 0; j < P; ++j) Rm[i][j] = Rg[i * P + j];
    ld_vec<P>(static_cast<const R*>(a.yslot), st, cs, y);
    linearize_h<Model, R>(md, kTaylor, a.rule, Rm, x, Px, y, H, d, Rp, yt);
  }
  const R* filt = static_cast<const R*>(a.filt);
  R xf[N], Pf[N][N], mp[N], Pp[N][N];
  ld_vec<N>(filt, st, cp, xf);
  ld_sym<N>(filt + N * st, st, cp, Pf);
  mat_vec<N, N>(F, xf, mp);
  PKS_UNROLL for (int i = 0; i < N; ++i) mp[i] += c[i];
  sandwich_add<N, N>(F, Pf, Qp, Pp);
  R HP[P][N], Sm[P][P], v[P], diag[P];
  mat_mul<P, N, N>(H, Pp, HP);
  PKS_UNROLL for (int i = 0; i < P; ++i)
    PKS_UNROLL for (int j = i; j < P; ++j) {
      R sum = Rp[i][j];
      PKS_UNROLL for (int t = 0; t < N; ++t) sum += HP[i][t] * H[j][t];
      Sm[i][j] = sum;
      Sm[j][i] = sum;
    }
  const bool ok = chol_inplace<P>(Sm, diag);
  PKS_UNROLL for (int i = 0; i < P; ++i) {
    R sum = yt[i] - d[i];
    PKS_UNROLL for (int t = 0; t < N; ++t) sum -= H[i][t] * mp[t];
    v[i] = sum;
  }
  chol_fwd_vec<P>(Sm, v);
  double quad = 0.0, logdet = 0.0;
  PKS_UNROLL for (int i = 0; i < P; ++i) {
    quad += double(v[i]) * double(v[i]);
    logdet += 2.0 * log(double(diag[i]));
  }
  constexpr double kLog2Pi = 1.8378770664093454836;
  a.slot_ll[s] = ok ? -0.5 * (P * kLog2Pi + logdet + quad) : __builtin_nan("");
}

// Puts back the saved trajectory (all `words` rows) at the slots of the tracks
// whose damped step was not taken.
template <typename R>
__global__ __launch_bounds__(kSlotBlock) void k_restore_tracks(int64_t S, size_t stride, SlotMap map, int words,
                                                               const int* track, const unsigned char* reject,
                                                               const R* saved, R* traj) {
  const int64_t cs = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  const int64_t s = map.slot(cs);
  if (s >= S || !reject[track[s]]) return;
  for (int w = 0; w < words; ++w) traj[size_t(w) * stride + cs] = saved[size_t(w) * stride + cs];
}

}  // namespace pks
