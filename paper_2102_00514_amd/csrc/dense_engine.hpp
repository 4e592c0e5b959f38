// Host side of the wavefront-cooperative path (dense.hpp): device memory plan,
// the kernel sequence of one iteration and its HIP graph.
//
// Scan hierarchy: level 0 folds `fan0` consecutive slots per wave; every
// higher level folds pairs of aggregates of the level below (fours for the
// smoothing scan), until at most that many remain; a single wave then scans
// those, and the down-sweeps hand exclusive carries back level by level.  Pairs
// keep the critical path of the upper levels at one operator per level: there a
// level has too few waves to fill the chip, and a fan of f would cost f - 1
// dependent combines instead.  The smoothing combine is about a quarter of the
// filtering one, so there fewer levels (fewer launches) win.
#pragma once

#include <algorithm>
#include <vector>

#include "dense.hpp"
#include "engine_base.hpp"
#include "objective.hpp"
#include "slot_kernels.hpp"

namespace pks {

template <class Model, typename R>
class DenseEngine final : public EngineBase {
 public:
  static constexpr int N = Model::N, P = Model::P;
  using Lay = dn::Layout<N, P>;
  static constexpr int kFan = 8;        // level 0: slots per wave (default)
  static constexpr int kLevelFan = 2;   // higher levels: aggregates per wave
  static constexpr int kLevelFanS = 4;  // the same for the smoothing scan, whose combine is 4x cheaper

  sm_status setup(const sm_problem& pb, hipStream_t st) override {
    stream = st;
    if (pb.lin == SM_LIN_TAYLOR) return fail(SM_EINVAL, "the full-state engine takes sigma-point linearisations");
    cap = pb.max_device_bytes;
    ntracks = pb.n_tracks;
    n_iter = pb.n_iter;
    lin_ = pb.lin;
    lm_ = pb.lm_lambda;
    rule_.alpha = pb.ut_alpha;
    rule_.kappa = pb.ut_kappa;
    use_graph_ = pb.use_graph != 0;
    const int64_t nmeas = pb.offsets[ntracks];
    S = nmeas + ntracks;
    fan0_ = pb.lane_slots >= 1 ? pb.lane_slots : kFan;
    sched_lanes = dn::kWave;
    sched_slots = fan0_;
    // scan levels
    int64_t c = (S + fan0_ - 1) / fan0_;
    counts_.push_back(c);
    while (c > kLevelFan) {
      c = (c + kLevelFan - 1) / kLevelFan;
      counts_.push_back(c);
    }
    c = counts_[0];
    counts_s_.push_back(c);
    while (c > kLevelFanS) {
      c = (c + kLevelFanS - 1) / kLevelFanS;
      counts_s_.push_back(c);
    }
    sched_tiles = counts_[0];
    // host-side tables
    std::vector<unsigned char> flags(S, 0);
    std::vector<int> track(S, 0);
    std::vector<R> ys(size_t(S) * P, R(0));
    int64_t s = 0;
    for (int i = 0; i < ntracks; ++i) {
      const int64_t T = pb.offsets[i + 1] - pb.offsets[i];
      for (int64_t k = 0; k <= T; ++k, ++s) {
        track[s] = i;
        flags[s] = (k == 0 ? kSlotFirst : 0u) | (k == T ? kSlotLast : 0u);
        if (k > 0)
          for (int q = 0; q < P; ++q) ys[size_t(s) * P + q] = R(pb.y[size_t(pb.offsets[i] + k - 1) * P + q]);
      }
    }
    auto cast = [](const double* p, size_t n) { return std::vector<R>(p, p + n); };
    const std::vector<R> prm = cast(pb.params, size_t(pb.n_params)), Q = cast(pb.Q, size_t(N) * N),
                         Rm = cast(pb.R, size_t(P) * P), m0 = cast(pb.m0, size_t(ntracks) * N),
                         P0 = cast(pb.P0, size_t(ntracks) * N * N);
    hipError_t e = hipSuccess;
    auto A = [&](void** p, size_t bytes) {
      if (e == hipSuccess) e = dalloc(p, bytes);
    };
    A(reinterpret_cast<void**>(&d_flags_), S);
    A(reinterpret_cast<void**>(&d_track_), sizeof(int) * S);
    A(&d_params_, sizeof(R) * prm.size());
    A(&d_Q_, sizeof(R) * Q.size());
    A(&d_R_, sizeof(R) * Rm.size());
    A(reinterpret_cast<void**>(&d_params64_), sizeof(double) * size_t(pb.n_params));   // the linearisation's
    A(reinterpret_cast<void**>(&d_Q64_), sizeof(double) * N * N);                       // FP64 copies
    A(reinterpret_cast<void**>(&d_R64_), sizeof(double) * P * P);
    A(&d_m0_, sizeof(R) * m0.size());
    A(&d_P0_, sizeof(R) * P0.size());
    A(&d_y_, sizeof(R) * ys.size());
    A(&d_traj_, sizeof(R) * Lay::kTraj * S);
    A(&d_trans_, sizeof(R) * Lay::kTrans * S);
    A(&d_hlin_, sizeof(R) * Lay::kHlin * S);
    A(&d_elem_, sizeof(R) * Lay::kFElem * S);
    A(reinterpret_cast<void**>(&delta_bits), sizeof(unsigned long long) * (ntracks + 1));
    // whitening matrices of Q, R and each P0 for the MAP objective, slot
    // offsets of the tracks for the per-track sums
    std::vector<double> w(size_t(N) * N);
    std::vector<R> wq(size_t(N) * N), wr(size_t(P) * P), wp0(size_t(ntracks) * N * N);
    if (!whitening(pb.Q, N, w.data())) return fail(SM_EINVAL, "Q is not positive definite");
    std::copy(w.begin(), w.end(), wq.begin());
    w.resize(size_t(P) * P);
    if (!whitening(pb.R, P, w.data())) return fail(SM_EINVAL, "R is not positive definite");
    std::copy(w.begin(), w.end(), wr.begin());
    w.resize(size_t(N) * N);
    for (int t = 0; t < ntracks; ++t) {
      if (!whitening(pb.P0 + size_t(t) * N * N, N, w.data())) return fail(SM_EINVAL, "P0 is not positive definite");
      std::copy(w.begin(), w.end(), wp0.begin() + size_t(t) * N * N);
    }
    std::vector<int64_t> slot_off(ntracks + 1);
    for (int i = 0; i <= ntracks; ++i) slot_off[i] = pb.offsets[i] + i;
    longest_ = 0;
    for (int i = 0; i < ntracks; ++i) longest_ = std::max<int64_t>(longest_, slot_off[i + 1] - slot_off[i]);
    A(&d_wq_, sizeof(R) * wq.size());
    A(&d_wr_, sizeof(R) * wr.size());
    A(&d_wp0_, sizeof(R) * wp0.size());
    A(reinterpret_cast<void**>(&d_slot_off_), sizeof(int64_t) * (ntracks + 1));
    for (size_t l = 0; l < counts_.size(); ++l) {
      void *fa = nullptr, *fc = nullptr;
      A(&fa, sizeof(R) * Lay::kFElem * counts_[l]);
      A(&fc, sizeof(R) * Lay::kCarry * counts_[l]);
      fagg_.push_back(fa);
      fcar_.push_back(fc);
    }
    for (size_t l = 0; l < counts_s_.size(); ++l) {
      void *sa = nullptr, *sc = nullptr;
      A(&sa, sizeof(R) * Lay::kSElem * counts_s_[l]);
      A(&sc, sizeof(R) * Lay::kCarry * counts_s_[l]);
      sagg_.push_back(sa);
      scar_.push_back(sc);
    }
    if (e != hipSuccess)
      return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE,
                  hip_msg(e, "device allocation") + " (plan needs more than is available or allowed)");
    auto H2D = [&](void* dst, const void* src, size_t bytes) {
      if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    H2D(d_flags_, flags.data(), S);
    H2D(d_track_, track.data(), sizeof(int) * S);
    H2D(d_params_, prm.data(), sizeof(R) * prm.size());
    H2D(d_Q_, Q.data(), sizeof(R) * Q.size());
    H2D(d_R_, Rm.data(), sizeof(R) * Rm.size());
    H2D(d_params64_, pb.params, sizeof(double) * size_t(pb.n_params));
    H2D(d_Q64_, pb.Q, sizeof(double) * N * N);
    H2D(d_R64_, pb.R, sizeof(double) * P * P);
    H2D(d_m0_, m0.data(), sizeof(R) * m0.size());
    H2D(d_P0_, P0.data(), sizeof(R) * P0.size());
    H2D(d_y_, ys.data(), sizeof(R) * ys.size());
    H2D(d_wq_, wq.data(), sizeof(R) * wq.size());
    H2D(d_wr_, wr.data(), sizeof(R) * wr.size());
    H2D(d_wp0_, wp0.data(), sizeof(R) * wp0.size());
    H2D(d_slot_off_, slot_off.data(), sizeof(int64_t) * (ntracks + 1));
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "upload of the problem"));
    if (pb.init_mean) {
      std::vector<R> tj(size_t(S) * Lay::kTraj);
      for (int64_t sl = 0; sl < S; ++sl) {
        R* t = tj.data() + size_t(sl) * Lay::kTraj;
        for (int i = 0; i < N; ++i) t[i] = R(pb.init_mean[size_t(sl) * N + i]);
        const double* C = pb.init_cov ? pb.init_cov + size_t(sl) * N * N : pb.P0 + size_t(track[sl]) * N * N;
        for (int i = 0; i < N; ++i)
          for (int j = i; j < N; ++j) t[N + sym_index<N>(i, j)] = R(0.5 * (C[i * N + j] + C[j * N + i]));
      }
      H2D(d_traj_, tj.data(), sizeof(R) * tj.size());
    } else {
      const int64_t cnt = S * Lay::kTraj;
      hipLaunchKernelGGL((dn::k_dn_prior<N, R>), dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, stream, S,
                         static_cast<const int*>(d_track_), static_cast<const R*>(d_m0_),
                         static_cast<const R*>(d_P0_), static_cast<R*>(d_traj_));
    }
    hipLaunchKernelGGL(k_fill_u64, dim3((ntracks + 256) / 256), dim3(256), 0, stream, delta_bits,
                       int64_t(ntracks + 1), 0ull);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "initial trajectory"));
    return SM_OK;
  }

  dn::DnArgs args() const {
    dn::DnArgs a;
    a.S = S;
    a.ntracks = ntracks;
    a.lin = lin_;
    a.rule = rule_;
    a.lm = lm_;
    a.flags = d_flags_;
    a.track = d_track_;
    a.params = d_params_;
    a.Q = d_Q_;
    a.Rm = d_R_;
    a.params64 = d_params64_;
    a.Q64 = d_Q64_;
    a.Rm64 = d_R64_;
    a.m0 = d_m0_;
    a.P0 = d_P0_;
    a.y = d_y_;
    a.traj = d_traj_;
    a.trans = d_trans_;
    a.hlin = d_hlin_;
    a.elem = d_elem_;
    a.delta_bits = delta_bits;
    return a;
  }

  template <bool FILT>
  void scan_levels() {
    const dn::DnArgs a = args();
    std::vector<void*>& agg = FILT ? fagg_ : sagg_;
    std::vector<void*>& car = FILT ? fcar_ : scar_;
    const char* up = FILT ? "scan_up_filter" : "scan_up_smoother";
    const char* down = FILT ? "scan_down_filter" : "scan_down_smoother";
    const std::vector<int64_t>& counts = FILT ? counts_ : counts_s_;
    const int fan = FILT ? kLevelFan : kLevelFanS;
    const size_t top = counts.size() - 1;
    for (size_t l = 0; l < top; ++l) {
      const dn::DnLevel lv{agg[l], agg[l + 1], nullptr, nullptr, counts[l], fan};
      timed(up, counts[l], [&] {
        hipLaunchKernelGGL((dn::k_dn_scan_up<Model, FILT, R>), dim3(unsigned(counts[l + 1])), dim3(dn::kWave), 0,
                           stream, a, lv);
      });
    }
    for (size_t k = 0; k <= top; ++k) {
      const size_t l = top - k;
      const dn::DnLevel lv{agg[l], nullptr, car[l], l == top ? nullptr : car[l + 1], counts[l], fan};
      const unsigned grid = unsigned((counts[l] + fan - 1) / fan);
      timed(down, counts[l], [&] {
        hipLaunchKernelGGL((dn::k_dn_scan_down<Model, FILT, R>), dim3(grid), dim3(dn::kWave), 0, stream, a, lv);
      });
    }
  }

  void launch_iteration() {
    const dn::DnArgs a = args();
    const unsigned c0 = unsigned(counts_[0]);
    timed("reset_delta", ntracks + 1, [&] {
      hipLaunchKernelGGL(k_fill_u64, dim3((ntracks + 256) / 256), dim3(256), 0, stream, delta_bits,
                         int64_t(ntracks + 1), 0ull);
    });
    timed("dn_linearize", S, [&] {
      hipLaunchKernelGGL((dn::k_dn_linearize<Model, R>), dim3(unsigned(S)), dim3(dn::kWave), 0, stream, a);
    });
    timed("dn_forward_up", S, [&] {
      if (a.lm > 0.0)
        hipLaunchKernelGGL((dn::k_dn_forward_up<Model, R, true>), dim3(c0), dim3(dn::kWave), 0, stream, a, fan0_,
                           fagg_[0]);
      else
        hipLaunchKernelGGL((dn::k_dn_forward_up<Model, R, false>), dim3(c0), dim3(dn::kWave), 0, stream, a, fan0_,
                           fagg_[0]);
    });
    scan_levels<true>();
    // stores each slot's smoothing element over its filtering element: one launch even under repeats
    timed(
        "dn_forward_down_backward_up", S,
        [&] {
          hipLaunchKernelGGL((dn::k_dn_forward_down_backward_up<Model, R>), dim3(c0), dim3(dn::kWave), 0, stream, a,
                             fan0_, static_cast<const void*>(fcar_[0]), sagg_[0]);
        },
        false);
    scan_levels<false>();
    timed("dn_backward_down", S, [&] {
      hipLaunchKernelGGL((dn::k_dn_backward_down<Model, R>), dim3(c0), dim3(dn::kWave), 0, stream, a, fan0_,
                         static_cast<const void*>(scar_[0]));
    });
  }

  hipError_t capture_iteration() {
    hipError_t e = hipSuccess;
    if (!capture_stream_) e = hipStreamCreateWithFlags(&capture_stream_, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipStream_t user = stream;
    stream = capture_stream_;
    e = hipStreamBeginCapture(capture_stream_, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      launch_iteration();
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(capture_stream_, &g);
      if (e == hipSuccess) e = hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
    }
    stream = user;
    return e;
  }

  sm_status iterate(int k) override {
    for (int it = 0; it < k; ++it) {
      if (use_graph_ && !profiling) {
        if (!graph_exec_) {
          const hipError_t ge = capture_iteration();
          if (ge != hipSuccess) return fail(SM_EDEVICE, hip_msg(ge, "capture of the iteration graph"));
        }
        const hipError_t le = hipGraphLaunch(graph_exec_, stream);
        if (le != hipSuccess) return fail(SM_EDEVICE, hip_msg(le, "graph launch"));
      } else {
        launch_iteration();
      }
      ++iters;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "kernel launch"));
    return SM_OK;
  }

  sm_status result_host(double* mean, double* cov) override {
    std::vector<R> h(size_t(S) * Lay::kTraj);
    hipError_t e = hipMemcpyAsync(h.data(), d_traj_, sizeof(R) * h.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "copy of the result"));
    for (int64_t s = 0; s < S; ++s) {
      const R* t = h.data() + size_t(s) * Lay::kTraj;
      if (mean)
        for (int i = 0; i < N; ++i) mean[size_t(s) * N + i] = double(t[i]);
      if (cov)
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j) cov[(size_t(s) * N + i) * N + j] = double(t[N + sym_index<N>(i, j)]);
    }
    return SM_OK;
  }

  sm_status result_device(void* mean, void* cov) override {
    const int64_t cnt = S * N * N;
    hipLaunchKernelGGL((dn::k_dn_unpack<N, R>), dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, stream, S,
                       static_cast<const R*>(d_traj_), static_cast<R*>(mean), static_cast<R*>(cov));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "result kernel"));
    return SM_OK;
  }

  sm_status set_trajectory_device(const void* mean, const void* cov, const double* cov_const) override {
    SymConst<N, R> c{};
    if (cov_const)
      for (int i = 0; i < N; ++i)
        for (int j = i; j < N; ++j) c.v[sym_index<N>(i, j)] = R(0.5 * (cov_const[i * N + j] + cov_const[j * N + i]));
    const int64_t cnt = S * Lay::kTraj;
    hipLaunchKernelGGL((dn::k_dn_pack<N, R>), dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, stream, S,
                       static_cast<const R*>(mean), static_cast<const R*>(cov), c, cov_const ? 1 : 0,
                       static_cast<const int*>(d_track_), static_cast<const R*>(d_P0_), static_cast<R*>(d_traj_));
    hipLaunchKernelGGL(k_fill_u64, dim3((ntracks + 256) / 256), dim3(256), 0, stream, delta_bits,
                       int64_t(ntracks + 1), 0ull);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "trajectory kernels"));
    iters = 0;
    return SM_OK;
  }

  // per-slot and per-track double buffers of the objective and the
  // log-likelihood, allocated on first use
  sm_status ensure_sums() {
    if (d_slot_val_) return SM_OK;
    sum_chunks_ = int((longest_ + kSumChunk - 1) / kSumChunk);
    hipError_t e = dalloc(reinterpret_cast<void**>(&d_slot_val_), sizeof(double) * S);
    if (e == hipSuccess) e = dalloc(reinterpret_cast<void**>(&d_partial_), sizeof(double) * ntracks * sum_chunks_);
    if (e == hipSuccess) e = dalloc(reinterpret_cast<void**>(&d_track_val_), sizeof(double) * ntracks);
    if (e != hipSuccess) {
      d_slot_val_ = nullptr;
      return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, hip_msg(e, "per-track sum buffers"));
    }
    return SM_OK;
  }

  // per-slot values (queued) -> per-track sums in a fixed order -> host
  sm_status track_sums(double* out, const char* what) {
    hipLaunchKernelGGL(k_track_partials, dim3(unsigned(ntracks), unsigned(sum_chunks_)), dim3(kTrackSumB), 0, stream,
                       static_cast<const double*>(d_slot_val_), static_cast<const int64_t*>(d_slot_off_), ntracks,
                       d_partial_);
    hipLaunchKernelGGL(k_track_totals, dim3(unsigned((ntracks + kTrackSumB - 1) / kTrackSumB)), dim3(kTrackSumB), 0,
                       stream, static_cast<const double*>(d_partial_), ntracks, sum_chunks_, d_track_val_);
    std::vector<double> h(ntracks);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d_track_val_, sizeof(double) * ntracks, hipMemcpyDeviceToHost,
                                            stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, what));
    if (out) std::copy(h.begin(), h.end(), out);
    return SM_OK;
  }

  // MAP objective (Section 3) of the current trajectory per track: one lane
  // per slot on the slot-major records.
  sm_status objective(double* out) override {
    sm_status st = ensure_sums();
    if (st != SM_OK) return st;
    CostArgs a{};
    a.S = S;
    a.stride = 1;
    a.ntracks = ntracks;
    a.flags = d_flags_;
    a.track = d_track_;
    a.params = d_params_;
    a.m0 = d_m0_;
    a.yslot = d_y_;
    a.traj = d_traj_;
    a.wq = d_wq_;
    a.wr = d_wr_;
    a.wp0 = d_wp0_;
    a.slot_cost = d_slot_val_;
    a.map = SlotMap{64, 1};
    a.traj_scale = Lay::kTraj;
    a.y_scale = P;
    a.m0_stride = 1;
    a.m0_scale = N;
    hipLaunchKernelGGL((k_objective_slots<Model, R>), dim3(unsigned((S + kSlotBlock - 1) / kSlotBlock)),
                       dim3(kSlotBlock), 0, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "objective"));
    return track_sums(out, "objective");
  }

  // One filtering pass at the current trajectory without damping: the
  // linearisation and the filtering half of an iteration, the filtered
  // moments of every slot, and log p(y_{1:T}) of the linearised model per
  // track.  The trajectory and the change statistics are left as they are.
  sm_status filter(double* mean, double* cov, double* loglik) override {
    sm_status st = ensure_sums();
    if (st != SM_OK) return st;
    hipError_t e = hipSuccess;
    if (!d_filt_) e = dalloc(&d_filt_, sizeof(R) * Lay::kTraj * S);
    if (e != hipSuccess)
      return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, hip_msg(e, "filtering pass buffers"));
    dn::DnArgs a = args();
    a.lm = 0.0;
    const unsigned c0 = unsigned(counts_[0]);
    hipLaunchKernelGGL((dn::k_dn_linearize<Model, R>), dim3(unsigned(S)), dim3(dn::kWave), 0, stream, a);
    hipLaunchKernelGGL((dn::k_dn_forward_up<Model, R, false>), dim3(c0), dim3(dn::kWave), 0, stream, a, fan0_,
                       fagg_[0]);   // a.lm is 0 here
    const double lm_saved = lm_;
    lm_ = 0.0;                       // the scan levels take their arguments from args()
    scan_levels<true>();
    lm_ = lm_saved;
    hipLaunchKernelGGL((dn::k_dn_forward_down_filter<Model, R>), dim3(c0), dim3(dn::kWave), 0, stream, a, fan0_,
                       static_cast<const void*>(fcar_[0]), d_filt_);
    hipLaunchKernelGGL((dn::k_dn_loglik<Model, R>), dim3(unsigned(S)), dim3(dn::kWave), 0, stream, a,
                       static_cast<const void*>(d_filt_), d_slot_val_);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "filtering pass"));
    st = track_sums(loglik, "log-likelihood");
    if (st != SM_OK || (!mean && !cov)) return st;
    std::vector<R> h(size_t(S) * Lay::kTraj);
    e = hipMemcpyAsync(h.data(), d_filt_, sizeof(R) * h.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "copy of the filtered moments"));
    for (int64_t sl = 0; sl < S; ++sl) {
      const R* t = h.data() + size_t(sl) * Lay::kTraj;
      if (mean)
        for (int i = 0; i < N; ++i) mean[size_t(sl) * N + i] = double(t[i]);
      if (cov)
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j) cov[(size_t(sl) * N + i) * N + j] = double(t[N + sym_index<N>(i, j)]);
    }
    return SM_OK;
  }

  ~DenseEngine() override {
    if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
    if (capture_stream_) (void)hipStreamDestroy(capture_stream_);
  }

 private:
  int lin_ = 0;
  SigmaRule rule_{1.0, 1.0};
  double lm_ = 0.0;
  bool use_graph_ = false;
  int fan0_ = kFan;
  hipGraphExec_t graph_exec_ = nullptr;
  hipStream_t capture_stream_ = nullptr;
  std::vector<int64_t> counts_, counts_s_;   // chunks per scan level (filtering, smoothing)
  std::vector<void*> fagg_, fcar_, sagg_, scar_;
  unsigned char* d_flags_ = nullptr;
  int* d_track_ = nullptr;
  void *d_params_ = nullptr, *d_Q_ = nullptr, *d_R_ = nullptr, *d_m0_ = nullptr, *d_P0_ = nullptr, *d_y_ = nullptr;
  double *d_params64_ = nullptr, *d_Q64_ = nullptr, *d_R64_ = nullptr;
  void *d_traj_ = nullptr, *d_trans_ = nullptr, *d_hlin_ = nullptr, *d_elem_ = nullptr;
  void *d_wq_ = nullptr, *d_wr_ = nullptr, *d_wp0_ = nullptr, *d_filt_ = nullptr;
  int64_t* d_slot_off_ = nullptr;
  int64_t longest_ = 0;
  int sum_chunks_ = 1;
  double *d_slot_val_ = nullptr, *d_partial_ = nullptr, *d_track_val_ = nullptr;
};

}  // namespace pks
