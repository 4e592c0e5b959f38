// One iteration of the method in three kernels over tiles of B lanes x K slots.
//
//   k_forward_up    build the filtering element of every slot (eq. 13-14) from
//                   its linearisation (Section 3: Taylor evaluated inline, or
//                   sigma-point regression read from a separate pass), fold
//                   each lane's K elements,
//                   Kogge-Stone over the lanes (eq. 15) -> lane prefixes
//                   (inclusive for K = 1, else exclusive with the elements
//                   stored) and the tile aggregate.
//   k_forward_down_backward_up
//                   apply the tile and lane carries to every slot -> filtered
//                   x*_k, P*_k; build the smoothing element (eq. 16-18); fold
//                   and ladder them in reverse slot order (eq. 19) -> reverse
//                   lane prefixes and tile aggregates.
//   k_backward_down apply the reverse carries -> smoothed xbar_k, Pbar_k,
//                   written in place, and the convergence statistic.
//
// Per-slot arrays use tile-transposed columns (SlotMap) so that, for each of
// a lane's K slots, a wavefront touches consecutive columns.
//
// Between them the tile aggregates are scanned into tile carries by a
// single-block scan (or the multi-level scan of scan.hpp for many tiles).
//
// The slot range is padded to tiles * B * K with single-slot dummy tracks
// (flags first|last, prior element (0, 0, I, 0, 0), end element (0, 0, I));
// padding never mixes with real tracks because of the reset property of the
// prior and end elements.  With the padded layout the forward tile t is the
// reverse tile tiles-1-t and forward lane l is reverse lane B-1-l, so the
// reverse scan runs over exactly the same slots as the forward one.
#pragma once

#include "elements.hpp"
#include "operators.hpp"
#include "scan.hpp"
#include "sqrt.hpp"

namespace pks {

enum : unsigned { kSlotFirst = 1u, kSlotLast = 2u, kSlotFrozen = 4u };

// Column of slot s in the per-slot arrays.  A tile of B lanes x K slots
// stores the j-th of lane l's K consecutive slots at column
// tile * B * K + j * B + l: for each j the lanes of a wavefront touch
// consecutive columns (coalesced), and every lane still owns a contiguous run
// of slots for its sequential fold.  K = 1 is the identity.
struct SlotMap {
  int B, K;
  PKS_HD int64_t col(int64_t s) const {
    if (K == 1) return s;
    const int64_t bk = int64_t(B) * K;
    const int64_t t = s / bk, r = s - t * bk;
    const int64_t l = r / K;
    return t * bk + (r - l * K) * B + l;
  }
  // inverse: the slot stored at column c (>= S for the padding of the last tile)
  PKS_HD int64_t slot(int64_t c) const {
    if (K == 1) return c;
    const int64_t bk = int64_t(B) * K;
    const int64_t t = c / bk, r = c - t * bk;
    const int64_t j = r / B;
    return t * bk + (r - j * B) * K + j;
  }
};

struct FusedArgs {
  int64_t S;            // real slots
  size_t stride;        // row stride of every slot array (>= padded slots)
  int K;                // slots per lane
  int64_t tiles;        // tiles of B*K slots
  int ntracks;
  const unsigned char* flags;
  const int* track;
  const void* params;
  const void* Q;        // N*N
  const void* R;        // P*P
  const void* m0;       // [N][ntracks]
  const void* P0;       // [s(N)][ntracks]
  const void* yslot;    // [P][stride]
  void* traj;           // [N + s(N)][stride]  xbar, Pbar (read by the forward kernel, updated in place at the end)
  const void* trans;    // sigma points: the linearisation pass's rows (LinLayout); Taylor: null
  void* selem;          // [SmootherOp words][stride] (K > 1)
  void* filt;           // optional [N + s(N)][stride]  x*, P*
  void *lx_f, *ta_f, *tc_f;  // forward lane exclusives [words][tiles*B], tile aggregates, tile carries
  void *lx_s, *ta_s, *tc_s;  // same for the reverse scan, indexed by reverse tile
  unsigned long long* delta_bits;  // [ntracks + 1]; entry ntracks = max over tracks
  SigmaRule rule;
  double lm;            // Levenberg-Marquardt damping lambda (0 = undamped)
  const double* lm_track;  // optional [ntracks]: per-track damping, replaces lm
  const unsigned char* frozen;  // optional [ntracks]: 1 = the track has converged and is not iterated
  SlotMap map;          // slot -> column of the per-slot arrays
};

// Frozen tracks.  A track that has converged can be taken out of later
// iterations: its slots then hold the padding elements (0, 0, I, 0, 0) and
// (0, 0, I), which restart both scans like a prior and an end element, so the
// tracks around it are unaffected, and its trajectory is not written.  A tile
// whose slots all belong to frozen tracks is skipped by every kernel; its
// aggregates are those padding elements.
enum : int { kTileActive = 0, kTileMixed = 1, kTileFrozen = 2 };

PKS_DEV bool slot_frozen(const FusedArgs& a, int64_t s) { return a.frozen && s < a.S && a.frozen[a.track[s]]; }

// kTileActive / kTileMixed / kTileFrozen for the slots [lo, lo + n) (tracks
// are contiguous, so the range covers the tracks track[lo]..track[last]).
PKS_DEV int tile_freeze_state(const FusedArgs& a, int64_t lo, int64_t n) {
  if (!a.frozen) return kTileActive;
  const int64_t hi = (lo + n < a.S ? lo + n : a.S) - 1;
  if (lo > hi) return kTileFrozen;       // padding only
  bool any_frozen = false, any_active = false;
  for (int k = a.track[lo]; k <= a.track[hi]; ++k) {
    if (a.frozen[k]) any_frozen = true;
    else any_active = true;
  }
  return any_active ? (any_frozen ? kTileMixed : kTileActive) : kTileFrozen;
}

// Linearisation arrays written by the separate linearisation pass: transition
// out of the slot F (N*N), c (N), Q' (s(N)); measurement at the slot H (P*N),
// d (P), R' (s(P)), ytil (P).
template <int N, int P>
struct LinLayout {
  static constexpr int kF = 0;
  static constexpr int kc = kF + N * N;
  static constexpr int kQ = kc + N;
  static constexpr int kH = kQ + sym_size<N>();
  static constexpr int kd = kH + P * N;
  static constexpr int kR = kd + P;
  static constexpr int ky = kR + sym_size<P>();
  static constexpr int kWords = ky + P;
};

template <int N>
struct TransLayout {
  static constexpr int kF = 0, kc = N * N, kQ = N * N + N, kWords = N * N + N + sym_size<N>();
};

// Where the forward kernel takes each slot's linearisation from.
enum LinSource : int {
  kInlineTaylor = 0,  // Jacobians evaluated in the kernel; F, c, Q' stored for the smoothing elements
  kStoredLin = 1      // read from the arrays a separate linearisation pass wrote (sigma-point SLR)
};

// How the elements carry their covariance-like blocks: as matrices
// (operators.hpp, eq. 13-19 as printed) or as lower-triangular factors
// (sqrt.hpp).  Both forms use the same words per element and per carry.
enum : int { kFormCov = 0, kFormSqrt = 1 };

template <int FORM, int N, typename R, bool ISO>
struct Form;

template <int N, typename R, bool ISO>
struct Form<kFormCov, N, R, ISO> {
  using FOp = FilterOp<N, R, ISO>;
  using SOp = SmootherOp<N, R, ISO>;
  template <int P>
  static PKS_DEV bool element(const R (&F)[N][N], const R (&c)[N], const R (&Qp)[N][N], const R (&H)[P][N],
                              const R (&d)[P], const R (&Rp)[P][P], const R (&yt)[P], typename FOp::Elem& e) {
    return filter_element<N, P, R>(F, c, Qp, H, d, Rp, yt, e.A, e.b, e.C, e.eta, e.J);
  }
  // prior element (0, m0, P0, 0, 0)
  static PKS_DEV void prior(const R (&P0)[N][N], typename FOp::Elem& e) {
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) e.C[i][j] = P0[i][j];
  }
  static PKS_DEV bool smoother(const typename FOp::Carry& c, const R (&F)[N][N], const R (&cc)[N],
                               const R (&Qp)[N][N], typename SOp::Elem& se) {
    return smoother_element<N, R>(c.b, c.C, F, cc, Qp, se.E, se.g, se.L);
  }
  // end element (0, x*_T, P*_T)
  static PKS_DEV void last(const typename FOp::Carry& c, typename SOp::Elem& se) {
    set_zero<N>(se.E);
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      se.g[i] = c.b[i];
      PKS_UNROLL for (int k = 0; k < N; ++k) se.L[i][k] = c.C[i][k];
    }
  }
  // mean and packed covariance of a carry into a [N + s(N)] slot array
  static PKS_DEV void store_moments(R* p, size_t st, size_t i, const typename FOp::Carry& c) {
    FOp::store(p, st, i, c);
  }
  static PKS_DEV void store_moments(R* p, size_t st, size_t i, const typename SOp::Carry& c) {
    SOp::store(p, st, i, c);
  }
};

template <int N, typename R, bool ISO>
struct Form<kFormSqrt, N, R, ISO> {
  using FOp = SqrtFilterOp<N, R, ISO>;
  using SOp = SqrtSmootherOp<N, R, ISO>;
  template <int P>
  static PKS_DEV bool element(const R (&F)[N][N], const R (&c)[N], const R (&Qp)[N][N], const R (&H)[P][N],
                              const R (&d)[P], const R (&Rp)[P][P], const R (&yt)[P], typename FOp::Elem& e) {
    return sqrt_filter_element<N, P, R>(F, c, Qp, H, d, Rp, yt, e.A, e.b, e.U, e.eta, e.Z);
  }
  // prior element (0, m0, chol P0, 0, 0)
  static PKS_DEV void prior(const R (&P0)[N][N], typename FOp::Elem& e) {
    if (!chol_lower<N>(P0, e.U)) e.b[0] = quiet_nan<R>();
  }
  static PKS_DEV bool smoother(const typename FOp::Carry& c, const R (&F)[N][N], const R (&cc)[N],
                               const R (&Qp)[N][N], typename SOp::Elem& se) {
    return sqrt_smoother_element<N, R>(c.b, c.U, F, cc, Qp, se.E, se.g, se.D);
  }
  static PKS_DEV void last(const typename FOp::Carry& c, typename SOp::Elem& se) {
    set_zero<N>(se.E);
    PKS_UNROLL for (int i = 0; i < N; ++i) {
      se.g[i] = c.b[i];
      PKS_UNROLL for (int k = 0; k < N; ++k) se.D[i][k] = c.U[i][k];
    }
  }
  static PKS_DEV void store_moments(R* p, size_t st, size_t i, const typename FOp::Carry& c) {
    R P[N][N];
    tril_gram<N>(c.U, P);
    st_vec<N>(p, st, i, c.b);
    st_sym<N>(p + N * st, st, i, P);
  }
  static PKS_DEV void store_moments(R* p, size_t st, size_t i, const typename SOp::Carry& c) {
    R P[N][N];
    tril_gram<N>(c.D, P);
    st_vec<N>(p, st, i, c.g);
    st_sym<N>(p + N * st, st, i, P);
  }
};

// Levenberg-Marquardt damping of the element of real slot s towards the
// previous iterate stored in traj (the linearisation point of this iteration).
template <int N, typename R>
PKS_DEV bool lm_damp_slot(const FusedArgs& a, int64_t s, typename FilterOp<N, R>::Elem& e) {
  const double lam = a.lm_track ? a.lm_track[a.track[s]] : a.lm;
  if (!(lam > 0.0)) return true;
  R xb[N];
  ld_vec<N>(static_cast<const R*>(a.traj), a.stride, a.map.col(s), xb);
  const bool ok = lm_damp_element<N, R>(R(lam), xb, e.A, e.b, e.C, e.eta, e.J);
  if (!ok) e.b[0] = quiet_nan<R>();
  return ok;
}

// Surrogate transition out of the slot at column cs: F, c and Q' (eq. 10
// evaluated at the linearisation point for Taylor, else the rows the
// sigma-point linearisation pass stored).  Nothing of it is stored between the
// kernels: the down-sweep evaluates or reads it again.
template <class Model, int SRC, typename R>
PKS_DEV void transition_of(const FusedArgs& a, int64_t cs, R (&F)[Model::N][Model::N], R (&c)[Model::N],
                           R (&Qp)[Model::N][Model::N]) {
  constexpr int N = Model::N, P = Model::P;
  const size_t st = a.stride;
  if constexpr (SRC == kStoredLin) {
    using LL = LinLayout<N, P>;
    const R* lin = static_cast<const R*>(a.trans);
    ld_mat<N, N>(lin + LL::kF * st, st, cs, F);
    ld_vec<N>(lin + LL::kc * st, st, cs, c);
    ld_sym<N>(lin + LL::kQ * st, st, cs, Qp);
  } else {
    const Model md{static_cast<const R*>(a.params)};
    R xp[N], Pp[N][N], Qm[N][N];
    ld_vec<N>(static_cast<const R*>(a.traj), st, cs, xp);
    set_zero<N>(Pp);
    const R* Qg = static_cast<const R*>(a.Q);
    PKS_UNROLL for (int i = 0; i < N; ++i) PKS_UNROLL for (int j = 0; j < N; ++j) Qm[i][j] = Qg[i * N + j];
    linearize_f<Model, R>(md, kTaylor, a.rule, Qm, xp, Pp, F, c, Qp);
  }
}

// Prior element (0, m0, P0, 0, 0) of the first slot of a track, or the
// padding element (0, 0, I, 0, 0).
template <class Model, typename R, int FORM>
PKS_DEV void prior_element(const FusedArgs& a, int64_t s, typename Form<FORM, Model::N, R, true>::FOp::Elem& e,
                           bool pad = false) {
  constexpr int N = Model::N;
  using Fm = Form<FORM, N, R, true>;
  set_zero<N>(e.A);
  set_zero<N>(e.eta);
  R P0[N][N];
  if (s < a.S && !pad) {
    const int tr = a.track[s];
    ld_vec<N>(static_cast<const R*>(a.m0), size_t(a.ntracks), tr, e.b);
    ld_sym<N>(static_cast<const R*>(a.P0), size_t(a.ntracks), tr, P0);
  } else {
    set_zero<N>(e.b);
    set_zero<N>(P0);
    PKS_UNROLL for (int i = 0; i < N; ++i) P0[i][i] = R(1);
  }
  if constexpr (FORM == kFormCov) {
    set_zero<N>(e.J);
    Fm::prior(P0, e);
    if (s < a.S && !pad && (a.lm > 0.0 || a.lm_track)) lm_damp_slot<N, R>(a, s, e);
  } else {
    set_zero<N>(e.Z);
    Fm::prior(P0, e);
  }
}

// Filtering element of slot s (not the first of its track) from the
// surrogate transition (F, c, Q') into it.
template <class Model, int SRC, typename R, int FORM>
PKS_DEV void filter_element_with(const FusedArgs& a, int64_t s, const R (&F)[Model::N][Model::N],
                                 const R (&c)[Model::N], const R (&Qp)[Model::N][Model::N],
                                 typename Form<FORM, Model::N, R, true>::FOp::Elem& e) {
  constexpr int N = Model::N, P = Model::P;
  using Fm = Form<FORM, N, R, true>;
  const size_t st = a.stride;
  const int64_t cs = a.map.col(s);
  R H[P][N], d[P], Rp[P][P], yt[P];
  if constexpr (SRC == kStoredLin) {
    using LL = LinLayout<N, P>;
    const R* lin = static_cast<const R*>(a.trans);
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
  bool ok = Fm::template element<P>(F, c, Qp, H, d, Rp, yt, e);
  if constexpr (FORM == kFormCov) {
    if (a.lm > 0.0 || a.lm_track) ok = lm_damp_slot<N, R>(a, s, e) && ok;
  }
  if (!ok) e.b[0] = quiet_nan<R>();
}

// Filtering element of slot s.
template <class Model, int SRC, typename R, int FORM = kFormCov>
PKS_DEV void build_filter_element(const FusedArgs& a, int64_t s,
                                  typename Form<FORM, Model::N, R, true>::FOp::Elem& e) {
  constexpr int N = Model::N;
  const unsigned fl = s < a.S ? a.flags[s] : (kSlotFirst | kSlotLast);
  const bool fz = slot_frozen(a, s);
  if ((fl & kSlotFirst) || fz) {
    prior_element<Model, R, FORM>(a, s, e, fz);
    return;
  }
  R F[N][N], c[N], Qp[N][N];
  transition_of<Model, SRC, R>(a, a.map.col(s - 1), F, c, Qp);
  filter_element_with<Model, SRC, R, FORM>(a, s, F, c, Qp, e);
}

// A lane's walk over its K slots in a forward down-sweep (K > 1): the
// filtering element of every slot is built again (from the linearisation, as
// in the up-sweep) and applied to the running carry.  The transition out of
// each slot is kept for the next slot's element and handed to `visit` with
// the slot's filtered carry: visit(j, s, cs, carry, flags, F, c, Q').
template <class Model, int SRC, typename R, bool ISO, int FORM, class Visit>
PKS_DEV void walk_lane(const FusedArgs& a, int64_t base, int64_t cbase, int B,
                       typename Form<FORM, Model::N, R, ISO>::FOp::Carry& c, bool have, Visit&& visit) {
  constexpr int N = Model::N;
  using FOp = typename Form<FORM, N, R, ISO>::FOp;
  R Ft[N][N], ct[N], Qt[N][N];   // transition into the current slot, then out of it
  bool trans_ok = false;
  for (int j = 0; j < a.K; ++j) {
    const int64_t s = base + j, cs = cbase + int64_t(j) * B;
    unsigned fl = s < a.S ? a.flags[s] : (kSlotFirst | kSlotLast);
    if (slot_frozen(a, s)) fl = kSlotFirst | kSlotLast | kSlotFrozen;
    if (a.K > 1) {
      typename Form<FORM, N, R, true>::FOp::Elem e;
      if (fl & kSlotFirst) {
        prior_element<Model, R, FORM>(a, s, e, (fl & kSlotFrozen) != 0);
      } else {
        if (!trans_ok) transition_of<Model, SRC, R>(a, a.map.col(s - 1), Ft, ct, Qt);
        filter_element_with<Model, SRC, R, FORM>(a, s, Ft, ct, Qt, e);
      }
      if (have) {
        typename FOp::Carry n;
        FOp::apply(c, e, n);
        c = n;
      } else {
        FOp::to_carry(e, c);
        have = true;
      }
    }
    trans_ok = visit(j, s, cs, c, fl, Ft, ct, Qt);
  }
}

template <class Model, int SRC, int B, typename R, bool ISO = true, int FORM = kFormCov>
__global__ __launch_bounds__(B) void k_forward_up(FusedArgs a) {
  constexpr int N = Model::N;
  using Op = typename Form<FORM, N, R, ISO>::FOp;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t base = (tile * B + lane) * a.K;
  const int64_t cbase = tile * B * a.K + lane;   // column of slot base + j: cbase + j * B
  if (tile == 0)
    for (int i = lane; i <= a.ntracks; i += B) a.delta_bits[i] = 0ull;
  if (a.frozen) {
    __shared__ int s_state;
    if (lane == 0) s_state = tile_freeze_state(a, tile * B * a.K, int64_t(B) * a.K);
    __syncthreads();
    if (s_state == kTileFrozen) {
      // the tile's aggregate is the padding element; nothing else is read
      if (lane == B - 1) {
        typename Op::Elem e;
        prior_element<Model, R, FORM>(a, a.S, e, true);
        Op::store(static_cast<R*>(a.ta_f), size_t(a.tiles), tile, e);
      }
      return;
    }
  }
  typename Op::Elem acc;
  // each lane folds its K elements as they are built; the down-sweep builds
  // them again rather than reading them back
  build_filter_element<Model, SRC, R, FORM>(a, base, acc);
  for (int j = 1; j < a.K; ++j) {
    typename Op::Elem e, r;
    build_filter_element<Model, SRC, R, FORM>(a, base + j, e);
    Op::combine(acc, e, r);
    acc = r;
  }
  typename Op::Elem ex;
  bool has_ex;
  block_ladder<Op, B, true, R>(lds, acc, ex, has_ex, true, a.K > 1);
  // K = 1: the lane's inclusive prefix goes to the down-sweep, which then
  // needs neither the element nor a second carry application; K > 1: the
  // exclusive prefix, continued there over the rebuilt elements
  if (a.K == 1) Op::store(static_cast<R*>(a.lx_f), size_t(a.tiles) * B, tile * B + lane, acc);
  else if (has_ex) Op::store(static_cast<R*>(a.lx_f), size_t(a.tiles) * B, tile * B + lane, ex);
  if (lane == B - 1) Op::store(static_cast<R*>(a.ta_f), size_t(a.tiles), tile, acc);
}

// Carry at the start of a lane's run in a forward down-sweep: tile carry (x)
// the lane prefix handed over by k_forward_up (inclusive for K = 1, so the
// result is already the filtered moments of the lane's slot).
template <int N, int B, typename R, bool ISO, int FORM = kFormCov>
PKS_DEV void lane_filter_carry(const FusedArgs& a, int64_t tile, int lane,
                               typename Form<FORM, N, R, ISO>::FOp::Carry& c, bool& have) {
  using FOp = typename Form<FORM, N, R, ISO>::FOp;
  have = false;
  if (tile > 0) {
    FOp::load(static_cast<const R*>(a.tc_f), size_t(a.tiles), tile - 1, c);
    have = true;
  }
  if (a.K == 1 || lane > 0) {
    typename FOp::Elem p;
    FOp::load(static_cast<const R*>(a.lx_f), size_t(a.tiles) * B, tile * B + lane, p);
    if (have) {
      typename FOp::Carry n;
      FOp::apply(c, p, n);
      c = n;
    } else {
      FOp::to_carry(p, c);
      have = true;
    }
  }
}

template <class Model, int SRC, int B, typename R, bool ISO = true, int FORM = kFormCov>
__global__ __launch_bounds__(B) void k_forward_down_backward_up(FusedArgs a) {
  constexpr int N = Model::N;
  using Fm = Form<FORM, N, R, ISO>;
  using FOp = typename Fm::FOp;
  using SOp = typename Fm::SOp;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t base = (tile * B + lane) * a.K;
  const size_t st = a.stride;
  const int rl = B - 1 - lane;
  const int64_t rt = a.tiles - 1 - tile;
  if (a.frozen) {
    __shared__ int s_state;
    if (lane == 0) s_state = tile_freeze_state(a, tile * B * a.K, int64_t(B) * a.K);
    __syncthreads();
    if (s_state == kTileFrozen) {
      if (rl == B - 1) {
        typename SOp::Elem se;
        typename FOp::Carry pc;
        set_zero<N>(pc.b);
        typename FOp::Elem pe;
        prior_element<Model, R, FORM>(a, a.S, pe, true);
        FOp::to_carry(pe, pc);
        Fm::last(pc, se);
        SOp::store(static_cast<R*>(a.ta_s), size_t(a.tiles), rt, se);
      }
      return;
    }
  }
  typename FOp::Carry c;
  bool have;
  lane_filter_carry<N, B, R, ISO, FORM>(a, tile, lane, c, have);
  typename SOp::Elem sacc;
  const int64_t cbase = tile * B * a.K + lane;
  walk_lane<Model, SRC, R, ISO, FORM>(
      a, base, cbase, B, c, have,
      [&](int j, int64_t s, int64_t cs, const typename FOp::Carry& cj, unsigned fl, R(&F)[N][N], R(&cc)[N],
          R(&Qp)[N][N]) {
        if (a.filt && !(fl & kSlotFrozen)) Fm::store_moments(static_cast<R*>(a.filt), st, cs, cj);
        typename SOp::Elem se;
        bool loaded = false;
        if (fl & kSlotFrozen) {
          // padding end element (0, 0, I) in place of the frozen slot's
          typename FOp::Elem pe;
          typename FOp::Carry pc;
          prior_element<Model, R, FORM>(a, a.S, pe, true);
          FOp::to_carry(pe, pc);
          Fm::last(pc, se);
        } else if (fl & kSlotLast) {
          Fm::last(cj, se);
        } else {
          transition_of<Model, SRC, R>(a, cs, F, cc, Qp);
          loaded = true;
          const bool ok = Fm::smoother(cj, F, cc, Qp, se);
          if (!ok) se.g[0] = quiet_nan<R>();
        }
        if (a.K > 1) SOp::store(static_cast<R*>(a.selem), st, cs, se);
        // paper order: sacc covers earlier slots, so sacc <- sacc (x) se, i.e.
        // the scan-order combine with se first
        if (j == 0) {
          sacc = se;
        } else {
          typename SOp::Elem r;
          SOp::combine(se, sacc, r);
          sacc = r;
        }
        (void)s;
        return loaded;
      });
  typename SOp::Elem ex;
  bool has_ex;
  block_ladder<SOp, B, false, R>(lds, sacc, ex, has_ex, true, a.K > 1);
  // as in the forward direction: inclusive prefix for K = 1, exclusive otherwise
  if (a.K == 1) SOp::store(static_cast<R*>(a.lx_s), size_t(a.tiles) * B, rt * B + rl, sacc);
  else if (has_ex) SOp::store(static_cast<R*>(a.lx_s), size_t(a.tiles) * B, rt * B + rl, ex);
  if (rl == B - 1) SOp::store(static_cast<R*>(a.ta_s), size_t(a.tiles), rt, sacc);
}

// Filtering pass only: forward down-sweep that stores the filtered moments
// (x*, P*) of every slot (the prefix of the filtering elements, Section 2).
template <class Model, int SRC, int B, typename R, bool ISO = true, int FORM = kFormCov>
__global__ __launch_bounds__(B) void k_forward_down_filter(FusedArgs a) {
  constexpr int N = Model::N;
  using Fm = Form<FORM, N, R, ISO>;
  using FOp = typename Fm::FOp;
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t base = (tile * B + lane) * a.K;
  typename FOp::Carry c;
  bool have;
  lane_filter_carry<N, B, R, ISO, FORM>(a, tile, lane, c, have);
  const int64_t cbase = tile * B * a.K + lane;
  walk_lane<Model, SRC, R, ISO, FORM>(a, base, cbase, B, c, have,
                                      [&](int, int64_t, int64_t cs, const typename FOp::Carry& cj, unsigned,
                                          R(&)[N][N], R(&)[N], R(&)[N][N]) {
                                        Fm::store_moments(static_cast<R*>(a.filt), a.stride, cs, cj);
                                        return false;
                                      });
}

PKS_DEV unsigned long long order_bits(double v) {
  // non-negative doubles and NaN order like their bit patterns as unsigned
  return static_cast<unsigned long long>(__double_as_longlong(v == v ? v : __builtin_nan("")));
}

template <class Model, int B, typename R, bool ISO = true, int FORM = kFormCov>
__global__ __launch_bounds__(B) void k_backward_down(FusedArgs a) {
  constexpr int N = Model::N;
  using Fm = Form<FORM, N, R, ISO>;
  using SOp = typename Fm::SOp;
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t base = (tile * B + lane) * a.K;
  const int rl = B - 1 - lane;
  const int64_t rt = a.tiles - 1 - tile;
  const size_t st = a.stride;
  __shared__ unsigned long long s_max;
  __shared__ int s_track;  // track of every real slot of the block, or -1 if several
  __shared__ int s_state;
  if (lane == 0) {
    s_max = 0ull;
    const int64_t lo = tile * B * a.K;
    const int64_t hi = (lo + int64_t(B) * a.K < a.S ? lo + int64_t(B) * a.K : a.S) - 1;
    s_track = (lo <= hi && a.track[lo] == a.track[hi]) ? a.track[lo] : -1;
    s_state = tile_freeze_state(a, lo, int64_t(B) * a.K);
  }
  __syncthreads();
  if (s_state == kTileFrozen) return;
  typename SOp::Carry c;
  bool have = false;
  if (rt > 0) {
    SOp::load(static_cast<const R*>(a.tc_s), size_t(a.tiles), rt - 1, c);
    have = true;
  }
  if (a.K == 1 || rl > 0) {
    typename SOp::Elem ex;
    SOp::load(static_cast<const R*>(a.lx_s), size_t(a.tiles) * B, rt * B + rl, ex);
    if (have) {
      typename SOp::Carry n;
      SOp::apply(c, ex, n);
      c = n;
    } else {
      SOp::to_carry(ex, c);
      have = true;
    }
  }
  R* traj = static_cast<R*>(a.traj);
  unsigned long long lane_max = 0ull;
  const int64_t cbase = tile * B * a.K + lane;
  for (int j = a.K - 1; j >= 0; --j) {
    const int64_t s = base + j, cs = cbase + int64_t(j) * B;
    if (a.K > 1) {
      typename SOp::Elem e;
      SOp::load(static_cast<const R*>(a.selem), st, cs, e);
      if (have) {
        typename SOp::Carry n;
        SOp::apply(c, e, n);
        c = n;
      } else {
        SOp::to_carry(e, c);
        have = true;
      }
    }
    if (s < a.S && !slot_frozen(a, s)) {
      double m = 0.0;
      bool nan = false;
      PKS_UNROLL for (int i = 0; i < N; ++i) {
        const double dlt = fabs(double(c.g[i]) - double(traj[i * st + cs]));
        nan = nan || !(dlt == dlt);
        m = dlt > m ? dlt : m;
      }
      const unsigned long long b = order_bits(nan ? __builtin_nan("") : m);
      Fm::store_moments(traj, st, cs, c);
      if (s_track < 0) atomicMax(&a.delta_bits[a.track[s]], b);
      lane_max = b > lane_max ? b : lane_max;
    }
  }
  atomicMax(&s_max, lane_max);
  __syncthreads();
  if (lane == 0) {
    if (s_track >= 0) atomicMax(&a.delta_bits[s_track], s_max);
    atomicMax(&a.delta_bits[a.ntracks], s_max);
  }
}

}  // namespace pks
