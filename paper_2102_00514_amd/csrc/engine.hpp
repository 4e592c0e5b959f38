// The engine template: device memory plan and kernel launch sequence for one
// (model, nx, ny, precision).  Included only by the instantiation units.
//
// One handle owns a plan for a batch of tracks laid out slot by slot (tracks
// concatenated, padded to whole tiles) and queues every iteration on the
// caller's HIP stream as three fused kernels (fused.hpp):
//   linearise + filtering elements + forward up-sweep
//   single-block scan of the tile aggregates
//   forward down-sweep + smoothing elements + reverse up-sweep
//   single-block scan of the reverse tile aggregates
//   reverse down-sweep + convergence statistic.
// When the tile aggregates do not fit one block, they are scanned by the
// generic multi-level kernels of scan.hpp instead.
// Tracks need no segmentation in the scans: the prior element that opens each
// track has A = 0, eta = J = 0, and the end element that closes it has E = 0,
// so no prefix or suffix leaks across a track boundary (the parts that do
// cross -- A, eta, J of a filtering prefix -- never reach the outputs).
#pragma once

#include <limits>
#include <memory>

#include "engine_base.hpp"
#include "objective.hpp"
#include "scan.hpp"
#include "slot_kernels.hpp"

namespace pks {

constexpr int kScanB = 64;        // lanes per scan tile (one wavefront)
constexpr int kLevelK = 2;        // positions per lane below the top level
constexpr int kTopMaxK = 8;       // a single block scans at most kTopB * kTopMaxK tile aggregates
constexpr int kTopB = 256;        // lanes of the single-block scan of the tile aggregates

struct ScanLevel {
  int64_t m;
  int K;
  int64_t tiles;
  void* lane_excl = nullptr;   // [elem words][tiles*B]
  void* tile_agg = nullptr;    // [elem words][tiles]
  void* tile_carry = nullptr;  // [carry words][tiles]
};

static std::vector<ScanLevel> plan_levels(int64_t S) {
  std::vector<ScanLevel> lv;
  int64_t m = S;
  while (m > int64_t(kScanB) * kTopMaxK) {
    ScanLevel L;
    L.m = m;
    L.K = kLevelK;
    L.tiles = (m + int64_t(kScanB) * kLevelK - 1) / (int64_t(kScanB) * kLevelK);
    lv.push_back(L);
    m = L.tiles;
  }
  ScanLevel top;
  top.m = m;
  top.K = int((m + kScanB - 1) / kScanB);
  top.tiles = 1;
  lv.push_back(top);
  return lv;
}

// Scan schedule: lanes per tile (B), slots per lane (K).
struct Schedule {
  int B = 256;
  int K = 1;
};

static Schedule choose_schedule(int64_t S, int lanes, int slots) {
  Schedule sc;
  if (lanes == 64 || lanes == 256) {
    sc.B = lanes;
  } else {
    sc.B = 256;
  }
  if (slots >= 1) {
    sc.K = slots;
  } else {
    // small problems: K = 1 keeps the dependent chain short; large ones fold
    // more slots per lane so fewer generic combines and tile aggregates occur
    sc.K = S <= int64_t(sc.B) * sc.B * 4 ? 1 : 4;
  }
  return sc;
}

template <class Model, typename R>
class Engine final : public EngineBase {
 public:
  static constexpr int N = Model::N, P = Model::P;
  static constexpr int kSN = sym_size<N>();
  static constexpr int kTrajW = N + kSN;
  using FOp = FilterOp<N, R>;
  using SOp = SmootherOp<N, R>;
  using LL = LinLayout<N, P>;
  using TL = TransLayout<N>;

  sm_status setup(const sm_problem& pb, hipStream_t st) override {
    stream = st;
    cap = pb.max_device_bytes;
    ntracks = pb.n_tracks;
    n_iter = pb.n_iter;
    lin_ = pb.lin;
    seq_ = pb.scan == SM_SCAN_SEQUENTIAL;
    // restart tests in the scan operators keep a failed track out of the
    // tracks after it; a single track has none after it
    iso_ = pb.n_tracks > 1;
    use_graph_ = pb.use_graph != 0 && !seq_;
    lm_ = pb.lm_lambda;
    form_ = pb.form;
    rule_.alpha = pb.ut_alpha;
    rule_.kappa = pb.ut_kappa;
    slot_off_.resize(ntracks + 1);
    for (int i = 0; i <= ntracks; ++i) slot_off_[i] = pb.offsets[i] + i;
    S = slot_off_[ntracks];
    sched_ = choose_schedule(S, pb.tile_lanes, pb.lane_slots);
    // the square-root form is compiled for 64-lane tiles with the restart
    // test (its operators are long; one instantiation keeps the build short)
    if (form_ == SM_FORM_SQRT) {
      sched_.B = 64;
      iso_ = true;
    }
    const int64_t per_tile = int64_t(sched_.B) * sched_.K;
    tiles_ = (S + per_tile - 1) / per_tile;
    const int64_t S_pad = tiles_ * per_tile;
    stride = size_t((S_pad + 63) / 64 * 64);
    top_single_ = tiles_ <= int64_t(kTopB) * kTopMaxK;
    sched_lanes = sched_.B;
    sched_slots = sched_.K;
    sched_tiles = tiles_;
    // the sequential path walks slots one lane per track: plain slot order
    map_ = SlotMap{sched_.B, seq_ ? 1 : sched_.K};
    std::vector<unsigned char> flags(S, 0);
    std::vector<int> track(S, 0);
    for (int i = 0; i < ntracks; ++i) {
      for (int64_t s = slot_off_[i]; s < slot_off_[i + 1]; ++s) track[s] = i;
      flags[slot_off_[i]] |= kSlotFirst;
      flags[slot_off_[i + 1] - 1] |= kSlotLast;
    }
    std::vector<R> prm(pb.params, pb.params + pb.n_params);
    std::vector<R> Q(pb.Q, pb.Q + N * N), Rm(pb.R, pb.R + P * P);
    std::vector<R> m0(size_t(N) * ntracks), P0(size_t(kSN) * ntracks);
    for (int t = 0; t < ntracks; ++t) {
      for (int i = 0; i < N; ++i) m0[size_t(i) * ntracks + t] = R(pb.m0[size_t(t) * N + i]);
      for (int i = 0; i < N; ++i)
        for (int j = i; j < N; ++j)
          P0[size_t(sym_index<N>(i, j)) * ntracks + t] = R(pb.P0[(size_t(t) * N + i) * N + j]);
    }
    // whitening matrices of Q, R and each P0 for the MAP objective
    std::vector<double> w(size_t(N) * N);
    std::vector<R> wq(size_t(N) * N), wr(size_t(P) * P), wp0(size_t(ntracks) * N * N);
    if (!whitening(pb.Q, N, w.data())) {
      if (pb.form != SM_FORM_SQRT) return fail(SM_EINVAL, "Q is not positive definite");
      // a positive semi-definite Q (factor form): the MAP objective, the only
      // user of this whitening, is refused for it
      std::fill(w.begin(), w.end(), std::numeric_limits<double>::quiet_NaN());
    }
    std::copy(w.begin(), w.end(), wq.begin());
    w.resize(size_t(P) * P);
    if (!whitening(pb.R, P, w.data())) return fail(SM_EINVAL, "R is not positive definite");
    std::copy(w.begin(), w.end(), wr.begin());
    w.resize(size_t(N) * N);
    for (int t = 0; t < ntracks; ++t) {
      if (!whitening(pb.P0 + size_t(t) * N * N, N, w.data())) return fail(SM_EINVAL, "P0 is not positive definite");
      std::copy(w.begin(), w.end(), wp0.begin() + size_t(t) * N * N);
    }
    std::vector<R> yslot(size_t(P) * stride, R(0));
    for (int t = 0; t < ntracks; ++t)
      for (int64_t k = 1; k < slot_off_[t + 1] - slot_off_[t]; ++k) {
        const int64_t s = slot_off_[t] + k, row = pb.offsets[t] + k - 1;
        for (int i = 0; i < P; ++i) yslot[size_t(i) * stride + map_.col(s)] = R(pb.y[row * P + i]);
      }
    // device plan
    hipError_t e = hipSuccess;
    auto A = [&](void** p, size_t bytes) {
      if (e == hipSuccess) e = dalloc(p, bytes);
    };
    A(&d_params_, sizeof(R) * std::max<size_t>(prm.size(), 1));
    A(&d_Q_, sizeof(R) * N * N);
    A(&d_R_, sizeof(R) * P * P);
    A(&d_m0_, sizeof(R) * m0.size());
    A(&d_P0_, sizeof(R) * P0.size());
    A(reinterpret_cast<void**>(&d_flags_), S);
    A(reinterpret_cast<void**>(&d_track_), sizeof(int) * S);
    A(reinterpret_cast<void**>(&d_slot_off_), sizeof(int64_t) * (ntracks + 1));
    A(&d_y_, sizeof(R) * yslot.size());
    A(&d_wq_, sizeof(R) * wq.size());
    A(&d_wr_, sizeof(R) * wr.size());
    A(&d_wp0_, sizeof(R) * wp0.size());
    A(&d_traj_[0], sizeof(R) * kTrajW * stride);
    A(reinterpret_cast<void**>(&delta_bits), sizeof(unsigned long long) * (ntracks + 1));
    if (seq_) {
      A(&d_traj_[1], sizeof(R) * kTrajW * stride);
      A(&d_lin_, sizeof(R) * LL::kWords * stride);
      A(&d_filt_, sizeof(R) * kTrajW * stride);
    } else {
      const size_t lanes = size_t(tiles_) * sched_.B;
      // Taylor transitions are evaluated again wherever they are needed; the
      // sigma-point linearisation runs as its own pass, whose arrays start with
      // the transition rows
      if (lin_ != SM_LIN_TAYLOR) {
        A(&d_lin_, sizeof(R) * LL::kWords * stride);
        d_trans_ = d_lin_;
      }
      // filtering elements are built again by the down-sweeps, never stored;
      // smoothing elements are stored for K > 1 (with one slot per lane the
      // reverse down-sweep starts from the lanes' inclusive prefixes)
      if (sched_.K > 1) A(&d_selem_, sizeof(R) * SOp::kElemWords * stride);
      // per-track freeze mask of smoother_iterate_until (all zero otherwise)
      if (ntracks > 1) A(reinterpret_cast<void**>(&d_frozen_), size_t(ntracks));
      A(&lx_f_, sizeof(R) * FOp::kElemWords * lanes);
      A(&ta_f_, sizeof(R) * FOp::kElemWords * tiles_);
      A(&tc_f_, sizeof(R) * FOp::kCarryWords * tiles_);
      A(&lx_s_, sizeof(R) * SOp::kElemWords * lanes);
      A(&ta_s_, sizeof(R) * SOp::kElemWords * tiles_);
      A(&tc_s_, sizeof(R) * SOp::kCarryWords * tiles_);
      if (!top_single_) {
        // generic multi-level scan of the tile aggregates
        levels_ = plan_levels(tiles_);
        for (size_t l = 0; l + 1 < levels_.size(); ++l) {
          ScanLevel& L = levels_[l];
          A(&L.lane_excl, sizeof(R) * FOp::kElemWords * L.tiles * kScanB);
          A(&L.tile_agg, sizeof(R) * FOp::kElemWords * L.tiles);
          A(&L.tile_carry, sizeof(R) * FOp::kCarryWords * L.tiles);
        }
      }
    }
    if (e != hipSuccess)
      return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE,
                  hip_msg(e, "device allocation") + " (plan needs more than is available or allowed)");
    e = set_lds_limits();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "kernel attributes"));
    auto H2D = [&](void* dst, const void* src, size_t bytes) {
      if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    };
    H2D(d_params_, prm.data(), sizeof(R) * prm.size());
    H2D(d_Q_, Q.data(), sizeof(R) * Q.size());
    H2D(d_R_, Rm.data(), sizeof(R) * Rm.size());
    H2D(d_m0_, m0.data(), sizeof(R) * m0.size());
    H2D(d_P0_, P0.data(), sizeof(R) * P0.size());
    H2D(d_flags_, flags.data(), S);
    H2D(d_track_, track.data(), sizeof(int) * S);
    H2D(d_slot_off_, slot_off_.data(), sizeof(int64_t) * (ntracks + 1));
    H2D(d_y_, yslot.data(), sizeof(R) * yslot.size());
    H2D(d_wq_, wq.data(), sizeof(R) * wq.size());
    H2D(d_wr_, wr.data(), sizeof(R) * wr.size());
    H2D(d_wp0_, wp0.data(), sizeof(R) * wp0.size());
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "upload of the problem"));
    const int64_t grid = (S + kSlotBlock - 1) / kSlotBlock;
    const SlotArgs a = slot_args(0);
    if (pb.init_mean) {
      std::vector<R> mean(pb.init_mean, pb.init_mean + size_t(S) * N);
      std::vector<R> cov(size_t(S) * N * N);
      for (int64_t s = 0; s < S; ++s)
        for (int i = 0; i < N * N; ++i)
          cov[size_t(s) * N * N + i] = R(pb.init_cov ? pb.init_cov[size_t(s) * N * N + i]
                                                     : pb.P0[size_t(track[s]) * N * N + i]);
      void *dm = nullptr, *dc = nullptr;
      e = hipMalloc(&dm, sizeof(R) * mean.size());
      if (e == hipSuccess) e = hipMalloc(&dc, sizeof(R) * cov.size());
      H2D(dm, mean.data(), sizeof(R) * mean.size());
      H2D(dc, cov.data(), sizeof(R) * cov.size());
      if (e == hipSuccess)
        hipLaunchKernelGGL((k_pack<N, R>), dim3(grid), dim3(kSlotBlock), 0, stream, S, stride, map_,
                           static_cast<const R*>(dm), static_cast<const R*>(dc), Place{N, 0},
                           static_cast<R*>(d_traj_[0]));
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (dm) (void)hipFree(dm);
      if (dc) (void)hipFree(dc);
      if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "upload of the initial trajectory"));
    } else {
      hipLaunchKernelGGL((k_broadcast_prior<N, R>), dim3(grid), dim3(kSlotBlock), 0, stream, a,
                         static_cast<R*>(d_traj_[0]));
    }
    hipLaunchKernelGGL(k_fill_u64, dim3((ntracks + 256) / 256), dim3(256), 0, stream, delta_bits,
                       int64_t(ntracks + 1), 0ull);
    e = hipGetLastError();
    if (e == hipSuccess && d_frozen_) e = hipMemsetAsync(d_frozen_, 0, size_t(ntracks), stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "initial trajectory"));
    cur_ = 0;
    return SM_OK;
  }

  // the ladders keep one element per wavefront in LDS
  size_t lds_filter() const { return sizeof(R) * FOp::kElemWords * (sched_.B / 64); }
  size_t lds_smoother() const { return sizeof(R) * SOp::kElemWords * (sched_.B / 64); }

  template <int B, bool ISO, int FORM>
  hipError_t set_lds_limits_b() {
    using Fm = Form<FORM, N, R, ISO>;
    hipError_t e = hipSuccess;
    auto set = [&](const void* f, size_t bytes) {
      if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    };
    set(reinterpret_cast<const void*>(&k_forward_up<Model, kInlineTaylor, B, R, ISO, FORM>), lds_filter());
    set(reinterpret_cast<const void*>(&k_forward_up<Model, kStoredLin, B, R, ISO, FORM>), lds_filter());
    set(reinterpret_cast<const void*>(&k_forward_down_backward_up<Model, kInlineTaylor, B, R, ISO, FORM>),
        lds_smoother());
    set(reinterpret_cast<const void*>(&k_forward_down_backward_up<Model, kStoredLin, B, R, ISO, FORM>),
        lds_smoother());
    set(reinterpret_cast<const void*>(&k_scan_single<typename Fm::FOp, kTopB, R>),
        sizeof(R) * FOp::kElemWords * (kTopB / 64));
    set(reinterpret_cast<const void*>(&k_scan_single<typename Fm::SOp, kTopB, R>),
        sizeof(R) * SOp::kElemWords * (kTopB / 64));
    return e;
  }

  template <int FORM>
  hipError_t set_lds_limits_f() {
    if constexpr (FORM == kFormSqrt) {
      return set_lds_limits_b<64, true, FORM>();
    } else {
      if (iso_) return sched_.B == 64 ? set_lds_limits_b<64, true, FORM>() : set_lds_limits_b<256, true, FORM>();
      return sched_.B == 64 ? set_lds_limits_b<64, false, FORM>() : set_lds_limits_b<256, false, FORM>();
    }
  }

  hipError_t set_lds_limits() {
    if (seq_) return hipSuccess;
    return form_ == SM_FORM_SQRT ? set_lds_limits_f<kFormSqrt>() : set_lds_limits_f<kFormCov>();
  }

  // grid of one lane per column of the per-slot arrays (padding included)
  dim3 col_grid() const {
    const int64_t cols = map_.K == 1 ? S : tiles_ * int64_t(sched_.B) * sched_.K;
    return dim3(unsigned((cols + kSlotBlock - 1) / kSlotBlock));
  }

  SlotArgs slot_args(int cur) const {
    SlotArgs a{};
    a.S = S;
    a.stride = stride;
    a.flags = d_flags_;
    a.track = d_track_;
    a.params = d_params_;
    a.Q = d_Q_;
    a.R = d_R_;
    a.m0 = d_m0_;
    a.P0 = d_P0_;
    a.tstride = size_t(ntracks);
    a.yslot = d_y_;
    a.traj = d_traj_[cur];
    a.lin = d_lin_;
    a.filt = d_filt_;
    a.traj_out = d_traj_[cur ^ 1];
    a.delta_bits = delta_bits;
    a.rule = rule_;
    a.lm = lm_;
    a.lm_track = lm_track_;
    a.frozen = d_frozen_;
    a.map = map_;
    return a;
  }

  FusedArgs fused_args() const {
    FusedArgs a{};
    a.S = S;
    a.stride = stride;
    a.K = sched_.K;
    a.tiles = tiles_;
    a.ntracks = ntracks;
    a.flags = d_flags_;
    a.track = d_track_;
    a.params = d_params_;
    a.Q = d_Q_;
    a.R = d_R_;
    a.m0 = d_m0_;
    a.P0 = d_P0_;
    a.yslot = d_y_;
    a.traj = d_traj_[0];
    a.trans = d_trans_;
    a.selem = d_selem_;
    a.filt = nullptr;
    a.lx_f = lx_f_;
    a.ta_f = ta_f_;
    a.tc_f = tc_f_;
    a.lx_s = lx_s_;
    a.ta_s = ta_s_;
    a.tc_s = tc_s_;
    a.delta_bits = delta_bits;
    a.rule = rule_;
    a.lm = lm_;
    a.lm_track = lm_track_;
    a.frozen = d_frozen_;
    a.map = map_;
    return a;
  }

  // Tracks taken out of (1) or put back into (0) the iterations; queued on the
  // stream (the mask is read by the kernels of the following iterations).
  sm_status set_frozen(const unsigned char* mask) override {
    if (!d_frozen_) return fail(SM_ESTATE, "freezing needs a batch on the parallel scan");
    if (!h_frozen_) {
      const hipError_t e = pinned_alloc(reinterpret_cast<void**>(&h_frozen_), size_t(ntracks));
      if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "freeze mask"));
    }
    // the previous upload may still be reading the pinned buffer
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) {
      if (mask) std::memcpy(h_frozen_, mask, size_t(ntracks));
      else std::memset(h_frozen_, 0, size_t(ntracks));
      e = hipMemcpyAsync(d_frozen_, h_frozen_, size_t(ntracks), hipMemcpyHostToDevice, stream);
    }
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "freeze mask upload"));
    return SM_OK;
  }
  bool can_freeze() const override { return d_frozen_ != nullptr; }

  // Generic multi-level scan of `m` elements stored in scan order (tile aggregates).
  template <class Op>
  void run_scan(const void* elems, int64_t m, void* out, const char* const (&names)[3]) {
    const size_t lds = sizeof(R) * Op::kElemWords * (kScanB / 64);
    const int L = int(levels_.size());
    for (int l = 0; l + 1 < L; ++l) {
      const ScanLevel& lv = levels_[l];
      ScanArgs a{};
      a.elems = l == 0 ? elems : levels_[l - 1].tile_agg;
      a.estride = l == 0 ? size_t(m) : size_t(levels_[l - 1].tiles);
      a.m = lv.m;
      a.K = lv.K;
      a.lane_excl = lv.lane_excl;
      a.lstride = size_t(lv.tiles) * kScanB;
      a.tile_agg = lv.tile_agg;
      a.tstride = size_t(lv.tiles);
      timed(names[0], lv.m, [&] {
        hipLaunchKernelGGL((k_scan_up<Op, kScanB, R>), dim3(lv.tiles), dim3(kScanB), lds, stream, a);
      });
    }
    {
      const ScanLevel& top = levels_[L - 1];
      ScanArgs a{};
      a.elems = L == 1 ? elems : levels_[L - 2].tile_agg;
      a.estride = L == 1 ? size_t(m) : size_t(levels_[L - 2].tiles);
      a.m = top.m;
      a.K = top.K;
      a.out = L == 1 ? out : levels_[L - 2].tile_carry;
      a.ostride = L == 1 ? size_t(m) : size_t(levels_[L - 2].tiles);
      timed(names[1], top.m, [&] {
        hipLaunchKernelGGL((k_scan_single<Op, kScanB, R>), dim3(1), dim3(kScanB), lds, stream, a);
      });
    }
    for (int l = L - 2; l >= 0; --l) {
      const ScanLevel& lv = levels_[l];
      ScanArgs a{};
      a.elems = l == 0 ? elems : levels_[l - 1].tile_agg;
      a.estride = l == 0 ? size_t(m) : size_t(levels_[l - 1].tiles);
      a.m = lv.m;
      a.K = lv.K;
      a.lane_excl = lv.lane_excl;
      a.lstride = size_t(lv.tiles) * kScanB;
      a.tile_carry = lv.tile_carry;
      a.cstride = size_t(lv.tiles);
      a.out = l == 0 ? out : levels_[l - 1].tile_carry;
      a.ostride = l == 0 ? size_t(m) : size_t(levels_[l - 1].tiles);
      timed(names[2], lv.m, [&] {
        hipLaunchKernelGGL((k_scan_down<Op, kScanB, R>), dim3(lv.tiles), dim3(kScanB), 0, stream, a);
      });
    }
  }

  // Tile aggregates -> inclusive tile carries: one 256-lane block when they fit,
  // the generic multi-level scan otherwise.
  template <class Op>
  void scan_tiles(void* agg, void* carry, const char* const (&names)[3]) {
    if (!top_single_) {
      run_scan<Op>(agg, tiles_, carry, names);
      return;
    }
    // tile t reads the inclusive carry of tiles 0..t-1, so the last tile's
    // aggregate is never needed: scan tiles_ - 1 positions (none for one tile)
    if (tiles_ < 2) return;
    ScanArgs a{};
    a.elems = agg;
    a.estride = size_t(tiles_);
    a.m = tiles_ - 1;
    a.out = carry;
    a.ostride = size_t(tiles_);
    timed(names[1], tiles_ - 1, [&] {
      hipLaunchKernelGGL((k_scan_single<Op, kTopB, R>), dim3(1), dim3(kTopB), sizeof(R) * Op::kElemWords * (kTopB / 64),
                         stream, a);
    });
  }

  template <int B, bool ISO, int FORM>
  void launch_iteration(const FusedArgs& a) {
    using Fm = Form<FORM, N, R, ISO>;
    static const char* const kFilterNames[3] = {"tiles_up_filter", "tiles_top_filter", "tiles_down_filter"};
    static const char* const kSmootherNames[3] = {"tiles_up_smoother", "tiles_top_smoother",
                                                  "tiles_down_smoother"};
    const dim3 grid{unsigned(tiles_)}, block{unsigned(B)};
    if (lin_ == SM_LIN_TAYLOR) {
      timed("forward_up", S, [&] {
        hipLaunchKernelGGL((k_forward_up<Model, kInlineTaylor, B, R, ISO, FORM>), grid, block, lds_filter(), stream,
                           a);
      });
    } else {
      const dim3 sgrid = col_grid();
      const SlotArgs sa = slot_args(0);
      timed("linearize", S, [&] { launch_linearize(sa, sgrid); });
      timed("forward_up", S, [&] {
        hipLaunchKernelGGL((k_forward_up<Model, kStoredLin, B, R, ISO, FORM>), grid, block, lds_filter(), stream, a);
      });
    }
    scan_tiles<typename Fm::FOp>(ta_f_, tc_f_, kFilterNames);
    timed("forward_down_backward_up", S, [&] {
      if (lin_ == SM_LIN_TAYLOR)
        hipLaunchKernelGGL((k_forward_down_backward_up<Model, kInlineTaylor, B, R, ISO, FORM>), grid, block,
                           lds_smoother(), stream, a);
      else
        hipLaunchKernelGGL((k_forward_down_backward_up<Model, kStoredLin, B, R, ISO, FORM>), grid, block,
                           lds_smoother(), stream, a);
    });
    scan_tiles<typename Fm::SOp>(ta_s_, tc_s_, kSmootherNames);
    timed("backward_down", S, [&] {
      hipLaunchKernelGGL((k_backward_down<Model, B, R, ISO, FORM>), grid, block, 0, stream, a);
    });
  }

  void launch_linearize(const SlotArgs& a, dim3 grid) {
    switch (lin_) {
      case SM_LIN_TAYLOR:
        hipLaunchKernelGGL((k_linearize<Model, kTaylor, R>), grid, dim3(kSlotBlock), 0, stream, a);
        break;
      case SM_LIN_CUBATURE:
        hipLaunchKernelGGL((k_linearize<Model, kCubature, R>), grid, dim3(kSlotBlock), 0, stream, a);
        break;
      default:
        hipLaunchKernelGGL((k_linearize<Model, kUnscented, R>), grid, dim3(kSlotBlock), 0, stream, a);
        break;
    }
  }

  sm_status iterate(int k) override {
    const dim3 grid(unsigned((S + kSlotBlock - 1) / kSlotBlock));
    for (int it = 0; it < k; ++it) {
      if (seq_) {
        const SlotArgs a = slot_args(cur_);
        timed("reset_delta", ntracks + 1, [&] {
          hipLaunchKernelGGL(k_fill_u64, dim3((ntracks + 256) / 256), dim3(256), 0, stream, delta_bits,
                             int64_t(ntracks + 1), 0ull);
        });
        timed("linearize", S, [&] { launch_linearize(a, grid); });
        timed("sequential", S, [&] {
          hipLaunchKernelGGL((k_sequential<N, P, R>), dim3((ntracks + 63) / 64), dim3(64), 0, stream, a,
                             d_slot_off_, ntracks);
        });
        timed("delta", S, [&] { hipLaunchKernelGGL((k_delta<N, R>), grid, dim3(kSlotBlock), 0, stream, a); });
        cur_ ^= 1;
      } else if (use_graph_ && !profiling) {
        if (!graph_exec_) {
          const hipError_t ge = capture_iteration();
          if (ge != hipSuccess) return fail(SM_EDEVICE, hip_msg(ge, "capture of the iteration graph"));
        }
        const hipError_t le = hipGraphLaunch(graph_exec_, stream);
        if (le != hipSuccess) return fail(SM_EDEVICE, hip_msg(le, "graph launch"));
      } else {
        launch_parallel_iteration();
      }
      ++iters;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "kernel launch"));
    return SM_OK;
  }

  template <int FORM>
  void launch_parallel_iteration_f(const FusedArgs& a) {
    if constexpr (FORM == kFormSqrt) {
      launch_iteration<64, true, FORM>(a);
    } else if (iso_) {
      if (sched_.B == 64) launch_iteration<64, true, FORM>(a);
      else launch_iteration<256, true, FORM>(a);
    } else {
      if (sched_.B == 64) launch_iteration<64, false, FORM>(a);
      else launch_iteration<256, false, FORM>(a);
    }
  }

  void launch_parallel_iteration() {
    const FusedArgs a = fused_args();
    if (form_ == SM_FORM_SQRT) launch_parallel_iteration_f<kFormSqrt>(a);
    else launch_parallel_iteration_f<kFormCov>(a);
  }

  // Records one iteration on a private stream (capture is not allowed on the
  // legacy default stream) and instantiates it; the kernels update the
  // trajectory in place and reset their own counters, so the same graph is
  // replayed for every iteration on the handle's stream.
  hipError_t capture_iteration() {
    hipError_t e = hipSuccess;
    if (!capture_stream_) e = hipStreamCreateWithFlags(&capture_stream_, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipStream_t user = stream;
    stream = capture_stream_;
    e = hipStreamBeginCapture(capture_stream_, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      launch_parallel_iteration();
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(capture_stream_, &g);
      if (e == hipSuccess) e = hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
    }
    stream = user;
    return e;
  }

  ~Engine() override {
    if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
    if (capture_stream_) (void)hipStreamDestroy(capture_stream_);
    for (void* p : pinned_) (void)hipHostFree(p);
  }

  // ---- MAP objective and Levenberg-Marquardt hooks ------------------------
  hipError_t pinned_alloc(void** p, size_t bytes) {
    const hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
    if (e == hipSuccess) pinned_.push_back(*p);
    return e;
  }

  // per-slot and per-track double buffers shared by the objective and the
  // log-likelihood, allocated on first use
  sm_status ensure_sums() {
    if (d_slot_cost_) return SM_OK;
    int64_t longest = 0;
    for (int t = 0; t < ntracks; ++t) longest = std::max<int64_t>(longest, slot_off_[t + 1] - slot_off_[t]);
    sum_chunks_ = int((longest + kSumChunk - 1) / kSumChunk);
    hipError_t e = dalloc(reinterpret_cast<void**>(&d_slot_cost_), sizeof(double) * S);
    if (e == hipSuccess) e = dalloc(reinterpret_cast<void**>(&d_partial_), sizeof(double) * ntracks * sum_chunks_);
    if (e == hipSuccess) e = dalloc(reinterpret_cast<void**>(&d_cost_), sizeof(double) * ntracks);
    if (e == hipSuccess) e = pinned_alloc(reinterpret_cast<void**>(&h_cost_), sizeof(double) * ntracks);
    if (e != hipSuccess) {
      d_slot_cost_ = nullptr;
      return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, hip_msg(e, "per-track sum buffers"));
    }
    return SM_OK;
  }

  // d_cost_ -> host, after the per-slot values have been queued
  sm_status track_sums_to_host(double* out, const char* what) {
    hipLaunchKernelGGL(k_track_partials, dim3(unsigned(ntracks), unsigned(sum_chunks_)), dim3(kTrackSumB), 0, stream,
                       static_cast<const double*>(d_slot_cost_), static_cast<const int64_t*>(d_slot_off_), ntracks,
                       d_partial_);
    hipLaunchKernelGGL(k_track_totals, dim3(unsigned((ntracks + kTrackSumB - 1) / kTrackSumB)), dim3(kTrackSumB), 0,
                       stream, static_cast<const double*>(d_partial_), ntracks, sum_chunks_, d_cost_);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h_cost_, d_cost_, sizeof(double) * ntracks, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, what));
    if (out) std::memcpy(out, h_cost_, sizeof(double) * ntracks);
    return SM_OK;
  }

  sm_status filter(double* mean, double* cov, double* loglik) override {
    sm_status st = ensure_sums();
    if (st != SM_OK) return st;
    hipError_t e = hipSuccess;
    if (!d_filt_) e = dalloc(&d_filt_, sizeof(R) * kTrajW * stride);
    if (e == hipSuccess && !d_delta_spare_)
      e = dalloc(reinterpret_cast<void**>(&d_delta_spare_), sizeof(unsigned long long) * (ntracks + 1));
    if (e != hipSuccess) {
      return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, hip_msg(e, "filtering pass buffers"));
    }
    const dim3 grid(unsigned((S + kSlotBlock - 1) / kSlotBlock));
    LoglikArgs la{};
    la.S = S;
    la.stride = stride;
    la.flags = d_flags_;
    la.params = d_params_;
    la.Q = d_Q_;
    la.R = d_R_;
    la.yslot = d_y_;
    la.traj = d_traj_[cur_];
    la.filt = d_filt_;
    la.rule = rule_;
    la.slot_ll = d_slot_cost_;
    la.map = map_;
    if (seq_) {
      // linearise, filter (the smoothed output goes to the spare trajectory
      // buffer and is discarded), then the predictive densities
      SlotArgs a = slot_args(cur_);
      a.lm = 0.0;
      a.lm_track = nullptr;
      launch_linearize(a, grid);
      hipLaunchKernelGGL((k_sequential<N, P, R>), dim3((ntracks + 63) / 64), dim3(64), 0, stream, a, d_slot_off_,
                         ntracks);
      la.trans = d_lin_;
      la.lin = d_lin_;
    } else {
      FusedArgs a = fused_args();
      a.lm = 0.0;
      a.lm_track = nullptr;
      a.frozen = nullptr;     // the filtering pass covers every track
      a.filt = d_filt_;
      a.delta_bits = d_delta_spare_;    // the forward kernel clears its statistic: keep the handle's
      if (form_ == SM_FORM_SQRT) launch_filter_pass_f<kFormSqrt>(a);
      else launch_filter_pass_f<kFormCov>(a);
      la.trans = d_trans_;            // null for Taylor: the density kernel evaluates the transition
      la.lin = lin_ == SM_LIN_TAYLOR ? nullptr : d_lin_;
    }
    hipLaunchKernelGGL((k_loglik_slots<Model, R>), col_grid(), dim3(kSlotBlock), 0, stream, la);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "filtering pass"));
    st = track_sums_to_host(loglik, "log-likelihood");
    if (st != SM_OK || (!mean && !cov)) return st;
    std::vector<R> h(size_t(kTrajW) * stride);
    e = hipMemcpyAsync(h.data(), d_filt_, sizeof(R) * h.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "copy of the filtered moments"));
    unpack_host(h, mean, cov);
    return SM_OK;
  }

  template <int FORM>
  void launch_filter_pass_f(const FusedArgs& a) {
    if constexpr (FORM == kFormSqrt) {
      launch_filter_pass<64, true, FORM>(a);
    } else if (iso_) {
      if (sched_.B == 64) launch_filter_pass<64, true, FORM>(a);
      else launch_filter_pass<256, true, FORM>(a);
    } else {
      if (sched_.B == 64) launch_filter_pass<64, false, FORM>(a);
      else launch_filter_pass<256, false, FORM>(a);
    }
  }

  template <int B, bool ISO, int FORM>
  void launch_filter_pass(const FusedArgs& a) {
    static const char* const kFilterNames[3] = {"tiles_up_filter", "tiles_top_filter", "tiles_down_filter"};
    const dim3 grid{unsigned(tiles_)}, block{unsigned(B)};
    if (lin_ == SM_LIN_TAYLOR) {
      hipLaunchKernelGGL((k_forward_up<Model, kInlineTaylor, B, R, ISO, FORM>), grid, block, lds_filter(), stream, a);
    } else {
      launch_linearize(slot_args(cur_), col_grid());
      hipLaunchKernelGGL((k_forward_up<Model, kStoredLin, B, R, ISO, FORM>), grid, block, lds_filter(), stream, a);
    }
    scan_tiles<typename Form<FORM, N, R, ISO>::FOp>(ta_f_, tc_f_, kFilterNames);
    if (lin_ == SM_LIN_TAYLOR)
      hipLaunchKernelGGL((k_forward_down_filter<Model, kInlineTaylor, B, R, ISO, FORM>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((k_forward_down_filter<Model, kStoredLin, B, R, ISO, FORM>), grid, block, 0, stream, a);
  }

  sm_status objective(double* out) override {
    const sm_status st = ensure_sums();
    if (st != SM_OK) return st;
    hipError_t e = hipSuccess;
    CostArgs a{};
    a.S = S;
    a.stride = stride;
    a.ntracks = ntracks;
    a.flags = d_flags_;
    a.track = d_track_;
    a.params = d_params_;
    a.m0 = d_m0_;
    a.yslot = d_y_;
    a.traj = d_traj_[cur_];
    a.wq = d_wq_;
    a.wr = d_wr_;
    a.wp0 = d_wp0_;
    a.slot_cost = d_slot_cost_;
    a.map = map_;
    a.traj_scale = 1;
    a.y_scale = 1;
    a.m0_stride = size_t(ntracks);
    a.m0_scale = 1;
    hipLaunchKernelGGL((k_objective_slots<Model, R>), col_grid(),
                       dim3(kSlotBlock), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "objective"));
    return track_sums_to_host(out, "objective");
  }

  sm_status lm_mode(bool on) override {
    if (on && form_ == SM_FORM_SQRT)
      return fail(SM_EINVAL, "adaptive damping is built for the covariance form of the elements");
    if (on && lin_ != SM_LIN_TAYLOR)
      return fail(SM_EINVAL, "adaptive damping needs the Taylor linearisation (sigma-point iterations minimise "
                             "no fixed objective)");
    if (on && !d_lam_) {
      hipError_t e = dalloc(reinterpret_cast<void**>(&d_lam_), sizeof(double) * ntracks);
      if (e == hipSuccess) e = dalloc(&d_saved_, sizeof(R) * kTrajW * stride);
      if (e == hipSuccess) e = dalloc(reinterpret_cast<void**>(&d_reject_), ntracks);
      if (e == hipSuccess) e = pinned_alloc(reinterpret_cast<void**>(&h_lam_), sizeof(double) * ntracks);
      if (e == hipSuccess) e = pinned_alloc(reinterpret_cast<void**>(&h_reject_), ntracks);
      if (e != hipSuccess) {
        d_lam_ = nullptr;
        return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, hip_msg(e, "damping buffers"));
      }
    }
    double* want = on ? d_lam_ : nullptr;
    if (want != lm_track_) {
      lm_track_ = want;
      // the captured iteration holds the kernel arguments: capture again
      if (graph_exec_) {
        const hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "stream before a new capture"));
        (void)hipGraphExecDestroy(graph_exec_);
        graph_exec_ = nullptr;
      }
    }
    return SM_OK;
  }

  sm_status lm_set_lambda(const double* lam) override {
    if (!lm_track_) return fail(SM_ESTATE, "adaptive damping is off");
    std::memcpy(h_lam_, lam, sizeof(double) * ntracks);
    const hipError_t e = hipMemcpyAsync(d_lam_, h_lam_, sizeof(double) * ntracks, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "damping upload"));
    return SM_OK;
  }

  sm_status lm_save() override {
    if (!lm_track_) return fail(SM_ESTATE, "adaptive damping is off");
    const hipError_t e =
        hipMemcpyAsync(d_saved_, d_traj_[cur_], sizeof(R) * kTrajW * stride, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "trajectory save"));
    return SM_OK;
  }

  sm_status lm_restore(const unsigned char* reject) override {
    if (!lm_track_) return fail(SM_ESTATE, "adaptive damping is off");
    std::memcpy(h_reject_, reject, ntracks);
    hipError_t e = hipMemcpyAsync(d_reject_, h_reject_, ntracks, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL((k_restore_tracks<R>), col_grid(), dim3(kSlotBlock),
                         0, stream, S, stride, map_, kTrajW, static_cast<const int*>(d_track_),
                         static_cast<const unsigned char*>(d_reject_), static_cast<const R*>(d_saved_),
                         static_cast<R*>(d_traj_[cur_]));
      e = hipGetLastError();
    }
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "trajectory restore"));
    return SM_OK;
  }

  sm_status result_host(double* mean, double* cov) override {
    std::vector<R> h(size_t(kTrajW) * stride);
    hipError_t e = hipMemcpyAsync(h.data(), d_traj_[cur_], sizeof(R) * h.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "copy of the result"));
    unpack_host(h, mean, cov);
    return SM_OK;
  }

  // slot-major host arrays (full symmetric covariances) from a [N + s(N)][stride] copy
  void unpack_host(const std::vector<R>& h, double* mean, double* cov) const {
    for (int64_t s = 0; s < S; ++s) {
      if (mean)
        for (int i = 0; i < N; ++i) mean[size_t(s) * N + i] = double(h[size_t(i) * stride + map_.col(s)]);
      if (cov)
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j)
            cov[(size_t(s) * N + i) * N + j] = double(h[size_t(N + sym_index<N>(i, j)) * stride + map_.col(s)]);
    }
  }

  sm_status result_device(void* mean, void* cov) override { return result_device_placed(mean, cov, N, 0); }

  sm_status result_device_placed(void* mean, void* cov, int ld, int off) override {
    const dim3 grid(unsigned((S + kSlotBlock - 1) / kSlotBlock));
    hipLaunchKernelGGL((k_unpack<N, R>), grid, dim3(kSlotBlock), 0, stream, S, stride, map_,
                       static_cast<const R*>(d_traj_[cur_]), static_cast<R*>(mean), static_cast<R*>(cov),
                       Place{ld, off});
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "result kernel"));
    return SM_OK;
  }

  sm_status set_trajectory_device(const void* mean, const void* cov, const double* cov_const) override {
    return set_trajectory_placed(mean, cov, cov_const, N, 0);
  }

  // cov_const, when used, is this engine's N x N block (row-major).
  sm_status set_trajectory_placed(const void* mean, const void* cov, const double* cov_const, int ld,
                                  int off) override {
    const dim3 grid(unsigned((S + kSlotBlock - 1) / kSlotBlock));
    R* traj = static_cast<R*>(d_traj_[cur_]);
    const R* m = static_cast<const R*>(mean);
    const Place pl{ld, off};
    if (cov) {
      hipLaunchKernelGGL((k_pack<N, R>), grid, dim3(kSlotBlock), 0, stream, S, stride, map_, m, static_cast<const R*>(cov),
                         pl, traj);
    } else if (cov_const) {
      SymConst<N, R> c;
      for (int i = 0; i < N; ++i)
        for (int j = i; j < N; ++j)
          c.v[sym_index<N>(i, j)] = R(0.5 * (cov_const[i * N + j] + cov_const[j * N + i]));
      hipLaunchKernelGGL((k_pack_const<N, R>), grid, dim3(kSlotBlock), 0, stream, S, stride, map_, m, pl, c, traj);
    } else {
      hipLaunchKernelGGL((k_broadcast_prior<N, R>), grid, dim3(kSlotBlock), 0, stream, slot_args(cur_), traj);
      hipLaunchKernelGGL((k_set_mean<N, R>), grid, dim3(kSlotBlock), 0, stream, S, stride, map_, m, pl, traj);
    }
    hipLaunchKernelGGL(k_fill_u64, dim3((ntracks + 256) / 256), dim3(256), 0, stream, delta_bits,
                       int64_t(ntracks + 1), 0ull);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "trajectory kernels"));
    iters = 0;
    return SM_OK;
  }

 private:
  int lin_ = 0;
  bool seq_ = false;
  bool iso_ = true;
  bool use_graph_ = false;
  hipGraphExec_t graph_exec_ = nullptr;
  hipStream_t capture_stream_ = nullptr;
  SigmaRule rule_{1.0, 1.0};
  double lm_ = 0.0;
  int form_ = SM_FORM_COVARIANCE;
  double* lm_track_ = nullptr;          // per-track damping while adaptive damping runs
  SlotMap map_{64, 1};                  // slot -> column of the per-slot arrays
  int cur_ = 0;
  Schedule sched_;
  int64_t tiles_ = 0;
  bool top_single_ = true;
  std::vector<int64_t> slot_off_;
  std::vector<ScanLevel> levels_;
  void *d_params_ = nullptr, *d_Q_ = nullptr, *d_R_ = nullptr, *d_m0_ = nullptr, *d_P0_ = nullptr;
  unsigned char* d_flags_ = nullptr;
  int* d_track_ = nullptr;
  int64_t* d_slot_off_ = nullptr;
  void *d_y_ = nullptr, *d_traj_[2] = {nullptr, nullptr};
  void *d_lin_ = nullptr, *d_filt_ = nullptr;  // sequential path
  void *d_wq_ = nullptr, *d_wr_ = nullptr, *d_wp0_ = nullptr;  // whitening of Q, R, P0
  double *d_slot_cost_ = nullptr, *d_cost_ = nullptr, *h_cost_ = nullptr, *d_partial_ = nullptr;
  int sum_chunks_ = 1;
  double *d_lam_ = nullptr, *h_lam_ = nullptr;
  void* d_saved_ = nullptr;
  unsigned char *d_reject_ = nullptr, *h_reject_ = nullptr;
  unsigned char *d_frozen_ = nullptr, *h_frozen_ = nullptr;   // per-track freeze mask (batches)
  unsigned long long* d_delta_spare_ = nullptr;   // statistic cleared by a filtering pass
  std::vector<void*> pinned_;
  void *d_trans_ = nullptr, *d_selem_ = nullptr;
  void *lx_f_ = nullptr, *ta_f_ = nullptr, *tc_f_ = nullptr, *lx_s_ = nullptr, *ta_s_ = nullptr, *tc_s_ = nullptr;
};

}  // namespace pks
