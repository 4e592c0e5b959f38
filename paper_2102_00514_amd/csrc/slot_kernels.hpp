// Per-slot helper kernels and the sequential comparison path.
//
// Device layout (structure of arrays, entry-major, `stride` >= slots):
//   traj  [N + s(N)][stride]   xbar, Pbar (upper-packed) of an iterate
//   yslot [P][stride]          y_k at the slot of x_k (unused at first slots)
//   lin   [LinLayout::kWords][stride]   (sequential path only)
//         transition out of the slot: F (N*N), c (N), Q' (s(N))
//         measurement at the slot:    H (P*N), d (P), R' (s(P)), ytil (P)
// Slot flags: bit 0 = first slot of a track (x_0), bit 1 = last slot (x_T).
#pragma once

#include "fused.hpp"

namespace pks {

struct SlotArgs {
  int64_t S;
  size_t stride;
  const unsigned char* flags;
  const int* track;
  const void* params;   // model parameters
  const void* Q;        // N*N
  const void* R;        // P*P
  const void* m0;       // [N][ntracks]
  const void* P0;       // [s(N)][ntracks]
  size_t tstride;       // ntracks
  const void* yslot;
  const void* traj;     // current iterate
  void* lin;
  void* filt;
  void* traj_out;
  unsigned long long* delta_bits;  // [ntracks + 1]; last entry = max over tracks
  SigmaRule rule;
  double lm;            // Levenberg-Marquardt damping lambda (0 = undamped)
  const double* lm_track;  // optional [ntracks]: per-track damping, replaces lm
  const unsigned char* frozen;  // optional [ntracks]: tracks taken out of the iterations
  SlotMap map;          // slot -> column of the per-slot arrays
};

constexpr int kSlotBlock = 256;

// One lane per column of the per-slot arrays (coalesced), launched over the
// padded column range.
template <class Model, int LIN, typename R>
__global__ __launch_bounds__(kSlotBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_linearize(SlotArgs a) {
  constexpr int N = Model::N, P = Model::P;
  using LL = LinLayout<N, P>;
  const int64_t cs = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  const int64_t s = a.map.slot(cs);
  if (s >= a.S) return;
  if (a.frozen && a.frozen[a.track[s]]) return;   // not iterated: its rows stay as they are
  const unsigned fl = a.flags[s];
  const R* traj = static_cast<const R*>(a.traj);
  R* lin = static_cast<R*>(a.lin);
  const size_t st = a.stride;
  Model md{static_cast<const R*>(a.params)};
  R xb[N], Pb[N][N];
  ld_vec<N>(traj, st, cs, xb);
  if constexpr (LIN != kTaylor) ld_sym<N>(traj + N * st, st, cs, Pb);
  else set_zero<N>(Pb);
  if (!(fl & kSlotLast)) {
    R Qm[N][N], F[N][N], c[N], Qp[N][N];
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Qm[i][j] = static_cast<const R*>(a.Q)[i * N + j];
    const bool ok = linearize_f<Model, R>(md, LIN, a.rule, Qm, xb, Pb, F, c, Qp);
    if (!ok) c[0] = quiet_nan<R>();
    st_mat<N, N>(lin + LL::kF * st, st, cs, F);
    st_vec<N>(lin + LL::kc * st, st, cs, c);
    st_sym<N>(lin + LL::kQ * st, st, cs, Qp);
  }
  if (!(fl & kSlotFirst)) {
    R Rm[P][P], y[P], H[P][N], d[P], Rp[P][P], yt[P];
    PKS_UNROLL for (int i = 0; i < P; ++i) PKS_UNROLL for (int j = 0; j < P; ++j) Rm[i][j] = static_cast<const R*>(a.R)[i * P + j];
    ld_vec<P>(static_cast<const R*>(a.yslot), st, cs, y);
    const bool ok = linearize_h<Model, R>(md, LIN, a.rule, Rm, xb, Pb, y, H, d, Rp, yt);
    if (!ok) d[0] = quiet_nan<R>();
    st_mat<P, N>(lin + LL::kH * st, st, cs, H);
    st_vec<P>(lin + LL::kd * st, st, cs, d);
    st_sym<P>(lin + LL::kR * st, st, cs, Rp);
    st_vec<P>(lin + LL::ky * st, st, cs, yt);
  }
}

// Per-track and global max |xbar_new - xbar_old| (NaN wins).  A block whose
// slots all belong to one track reduces in LDS and issues one global atomic.
template <int N, typename R>
__global__ __launch_bounds__(kSlotBlock) void k_delta(SlotArgs a) {
  const int64_t base = int64_t(blockIdx.x) * kSlotBlock;
  const int64_t s = base + threadIdx.x;
  __shared__ unsigned long long blk;
  __shared__ int same_track;
  if (threadIdx.x == 0) {
    blk = 0ull;
    const int64_t last = (base + kSlotBlock <= a.S ? base + kSlotBlock : a.S) - 1;
    same_track = a.track[base] == a.track[last];
  }
  __syncthreads();
  unsigned long long b = 0ull;
  if (s < a.S) {
    const R* o = static_cast<const R*>(a.traj);
    const R* n = static_cast<const R*>(a.traj_out);
    double m = 0.0;
    bool nan = false;
    const int64_t cs = a.map.col(s);
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      const double d = fabs(double(n[i * a.stride + cs]) - double(o[i * a.stride + cs]));
      nan = nan || !(d == d);
      m = d > m ? d : m;
    }
    b = order_bits(nan ? __builtin_nan("") : m);
    if (!same_track) atomicMax(&a.delta_bits[a.track[s]], b);
  }
  atomicMax(&blk, b);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (same_track) atomicMax(&a.delta_bits[a.track[base]], blk);
    atomicMax(&a.delta_bits[a.tstride], blk);
  }
}

static __global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static __global__ void k_fill_u32(unsigned int* p, int64_t n, unsigned int v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Initial trajectory: the prior of each track broadcast over its slots.
template <int N, typename R>
__global__ __launch_bounds__(kSlotBlock) void k_broadcast_prior(SlotArgs a, R* traj) {
  const int64_t s = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  if (s >= a.S) return;
  const int tr = a.track[s];
  constexpr int W = N + sym_size<N>();
  const R* m0 = static_cast<const R*>(a.m0);
  const R* P0 = static_cast<const R*>(a.P0);
  const int64_t cs = a.map.col(s);
  PKS_UNROLL for (int i = 0; i < N; ++i) traj[i * a.stride + cs] = m0[i * a.tstride + tr];
  PKS_UNROLL for (int i = 0; i < W - N; ++i) traj[(N + i) * a.stride + cs] = P0[i * a.tstride + tr];
}

// Placement of an N-state block inside a caller's state of dimension ld:
// mean[s * ld + off + i], cov[(s * ld + off + i) * ld + off + j].
struct Place {
  int ld, off;
};

// Packed device trajectory -> caller layout: mean [S][ld], cov [S][ld][ld].
template <int N, typename R>
__global__ __launch_bounds__(kSlotBlock) void k_unpack(int64_t S, size_t stride, SlotMap map, const R* traj, R* mean,
                                                       R* cov, Place pl) {
  const int64_t s = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  if (s >= S) return;
  const int64_t row = s * pl.ld + pl.off, cs = map.col(s);
  if (mean) PKS_UNROLL for (int i = 0; i < N; ++i) mean[row + i] = traj[i * stride + cs];
  if (cov)
    PKS_UNROLL for (int i = 0; i < N; ++i)
      PKS_UNROLL for (int j = 0; j < N; ++j)
        cov[(row + i) * pl.ld + pl.off + j] = traj[(N + sym_index<N>(i, j)) * stride + cs];
}

// Caller layout -> packed device trajectory (initial trajectory given by the caller).
template <int N, typename R>
__global__ __launch_bounds__(kSlotBlock) void k_pack(int64_t S, size_t stride, SlotMap map, const R* mean, const R* cov,
                                                     Place pl, R* traj) {
  const int64_t s = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  if (s >= S) return;
  const int64_t row = s * pl.ld + pl.off, cs = map.col(s);
  PKS_UNROLL for (int i = 0; i < N; ++i) traj[i * stride + cs] = mean[row + i];
  PKS_UNROLL for (int i = 0; i < N; ++i)
    PKS_UNROLL for (int j = i; j < N; ++j)
      traj[(N + sym_index<N>(i, j)) * stride + cs] =
          R(0.5) * (cov[(row + i) * pl.ld + pl.off + j] + cov[(row + j) * pl.ld + pl.off + i]);
}

// A covariance shared by every slot, upper-packed in sym_index order (passed by value).
template <int N, typename R>
struct SymConst {
  R v[sym_size<N>()];
};

// Caller means (device, placed by pl) -> packed trajectory; the covariance of
// every slot is the constant c.
template <int N, typename R>
__global__ __launch_bounds__(kSlotBlock) void k_pack_const(int64_t S, size_t stride, SlotMap map, const R* mean,
                                                           Place pl, SymConst<N, R> c, R* traj) {
  const int64_t s = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  if (s >= S) return;
  const int64_t cs = map.col(s);
  PKS_UNROLL for (int i = 0; i < N; ++i) traj[i * stride + cs] = mean[s * pl.ld + pl.off + i];
  PKS_UNROLL for (int i = 0; i < sym_size<N>(); ++i) traj[(N + i) * stride + cs] = c.v[i];
}

// Caller means (device, placed by pl) -> the mean rows of the packed trajectory only.
template <int N, typename R>
__global__ __launch_bounds__(kSlotBlock) void k_set_mean(int64_t S, size_t stride, SlotMap map, const R* mean,
                                                         Place pl, R* traj) {
  const int64_t s = int64_t(blockIdx.x) * kSlotBlock + threadIdx.x;
  if (s >= S) return;
  const int64_t cs = map.col(s);
  PKS_UNROLL for (int i = 0; i < N; ++i) traj[i * stride + cs] = mean[s * pl.ld + pl.off + i];
}

// ---------------------------------------------------------------------------
// Sequential comparison path: one lane per track runs the Kalman filter and
// the RTS smoother over the same linearised model (the recursions the scans
// replace).
// ---------------------------------------------------------------------------
template <int N, int P, typename R>
__global__ __launch_bounds__(64) void k_sequential(SlotArgs a, const int64_t* slot_off, int ntracks) {
  using LL = LinLayout<N, P>;
  const int tr = blockIdx.x * 64 + threadIdx.x;
  if (tr >= ntracks) return;
  const size_t st = a.stride;
  const R* lin = static_cast<const R*>(a.lin);
  R* filt = static_cast<R*>(a.filt);
  R* out = static_cast<R*>(a.traj_out);
  const int64_t s0 = slot_off[tr], s1 = slot_off[tr + 1];
  R m[N], Pm[N][N];
  ld_vec<N>(static_cast<const R*>(a.m0), a.tstride, tr, m);
  ld_sym<N>(static_cast<const R*>(a.P0), a.tstride, tr, Pm);
  const R* traj = static_cast<const R*>(a.traj);
  const double lam = a.lm_track ? a.lm_track[tr] : a.lm;
  if (lam > 0.0) {
    R xb[N];
    ld_vec<N>(traj, st, a.map.col(s0), xb);
    if (!lm_damp_moments<N, R>(R(lam), xb, m, Pm)) m[0] = quiet_nan<R>();
  }
  st_vec<N>(filt, st, a.map.col(s0), m);
  st_sym<N>(filt + N * st, st, a.map.col(s0), Pm);
  for (int64_t s = s0 + 1; s < s1; ++s) {
    R F[N][N], c[N], Qp[N][N], H[P][N], d[P], Rp[P][P], yt[P];
    ld_mat<N, N>(lin + LL::kF * st, st, a.map.col(s - 1), F);
    ld_vec<N>(lin + LL::kc * st, st, a.map.col(s - 1), c);
    ld_sym<N>(lin + LL::kQ * st, st, a.map.col(s - 1), Qp);
    ld_mat<P, N>(lin + LL::kH * st, st, a.map.col(s), H);
    ld_vec<P>(lin + LL::kd * st, st, a.map.col(s), d);
    ld_sym<P>(lin + LL::kR * st, st, a.map.col(s), Rp);
    ld_vec<P>(lin + LL::ky * st, st, a.map.col(s), yt);
    // predict
    R mp[N], Pp[N][N];
    mat_vec<N, N>(F, m, mp);
    PKS_UNROLL for (int i = 0; i < N; ++i) mp[i] += c[i];
    sandwich_add<N, N>(F, Pm, Qp, Pp);
    // update through S = L L^T, Z = L^-1 H P-
    R Z[P][N], Sm[P][P], v[P];
    mat_mul<P, N, N>(H, Pp, Z);
    PKS_UNROLL for (int i = 0; i < P; ++i)
      PKS_UNROLL for (int j = i; j < P; ++j) {
        R sum = Rp[i][j];
        PKS_UNROLL for (int t = 0; t < N; ++t) sum += Z[i][t] * H[j][t];
        Sm[i][j] = sum;
        Sm[j][i] = sum;
      }
    const bool ok = chol_inplace<P>(Sm);
    PKS_UNROLL for (int i = 0; i < P; ++i) {
      R sum = yt[i] - d[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) sum -= H[i][t] * mp[t];
      v[i] = sum;
    }
    chol_fwd<P, N>(Sm, Z);
    chol_fwd_vec<P>(Sm, v);
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R sum = mp[i];
      PKS_UNROLL for (int t = 0; t < P; ++t) sum += Z[t][i] * v[t];
      m[i] = ok ? sum : quiet_nan<R>();
      PKS_UNROLL for (int j = i; j < N; ++j) {
        R q = Pp[i][j];
        PKS_UNROLL for (int t = 0; t < P; ++t) q -= Z[t][i] * Z[t][j];
        Pm[i][j] = q;
        Pm[j][i] = q;
      }
    }
    if (lam > 0.0) {
      R xb[N];
      ld_vec<N>(traj, st, a.map.col(s), xb);
      if (!lm_damp_moments<N, R>(R(lam), xb, m, Pm)) m[0] = quiet_nan<R>();
    }
    st_vec<N>(filt, st, a.map.col(s), m);
    st_sym<N>(filt + N * st, st, a.map.col(s), Pm);
  }
  // RTS: xbar_T = x*_T, then backwards
  R xs[N], Ps[N][N];
  PKS_UNROLL for (int i = 0; i < N; ++i) {
    xs[i] = m[i];
    PKS_UNROLL for (int j = 0; j < N; ++j) Ps[i][j] = Pm[i][j];
  }
  st_vec<N>(out, st, a.map.col(s1 - 1), xs);
  st_sym<N>(out + N * st, st, a.map.col(s1 - 1), Ps);
  for (int64_t s = s1 - 2; s >= s0; --s) {
    R F[N][N], c[N], Qp[N][N], xf[N], Pf[N][N];
    ld_mat<N, N>(lin + LL::kF * st, st, a.map.col(s), F);
    ld_vec<N>(lin + LL::kc * st, st, a.map.col(s), c);
    ld_sym<N>(lin + LL::kQ * st, st, a.map.col(s), Qp);
    ld_vec<N>(filt, st, a.map.col(s), xf);
    ld_sym<N>(filt + N * st, st, a.map.col(s), Pf);
    R E[N][N], g[N], L[N][N];
    const bool ok = smoother_element<N, R>(xf, Pf, F, c, Qp, E, g, L);
    // xbar_k = g + E xbar_{k+1},  Pbar_k = L + E Pbar_{k+1} E^T
    R nx[N], nP[N][N];
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      R sum = g[i];
      PKS_UNROLL for (int t = 0; t < N; ++t) sum += E[i][t] * xs[t];
      nx[i] = ok ? sum : quiet_nan<R>();
    }
    sandwich_add<N, N>(E, Ps, L, nP);
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      xs[i] = nx[i];
      PKS_UNROLL for (int j = 0; j < N; ++j) Ps[i][j] = nP[i][j];
    }
    st_vec<N>(out, st, a.map.col(s), xs);
    st_sym<N>(out + N * st, st, a.map.col(s), Ps);
  }
}

}  // namespace pks
