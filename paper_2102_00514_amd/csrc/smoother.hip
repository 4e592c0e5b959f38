// Host runtime and C ABI of the parallel iterated smoother (include/smoother.h).
//
// One handle owns a device memory plan for a batch of tracks laid out slot by
// slot (tracks concatenated) and queues every iteration on the caller's HIP
// stream:
//   linearise -> filtering elements -> prefix scan (eq. 15) -> smoothing
//   elements -> suffix scan (eq. 19) -> per-track convergence statistic.
// Tracks need no segmentation in the scans: the prior element that opens each
// track has A = 0, eta = J = 0, and the end element that closes it has E = 0,
// so no prefix or suffix leaks across a track boundary (the parts that do
// cross -- A, eta, J of a filtering prefix -- never reach the outputs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "smoother.h"
#include "scan.hpp"
#include "slot_kernels.hpp"

namespace pks {

constexpr int kScanB = 64;        // lanes per scan tile (one wavefront)
constexpr int kLevelK = 2;        // positions per lane below the top level
constexpr int kTopMaxK = 8;       // the top level is one tile of <= kScanB * kTopMaxK positions

static thread_local std::string g_init_error;

static std::string hip_msg(hipError_t e, const char* what) {
  return std::string(what) + ": " + hipGetErrorString(e);
}

// ---------------------------------------------------------------------------
// Host-side validation helpers (double precision, plain loops).
// ---------------------------------------------------------------------------
static bool host_spd(const double* A, int n, double* worst_asym = nullptr) {
  std::vector<double> L(size_t(n) * n, 0.0);
  double scale = 0.0;
  for (int i = 0; i < n * n; ++i) {
    if (!std::isfinite(A[i])) return false;
    scale = std::max(scale, std::fabs(A[i]));
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (std::fabs(A[i * n + j] - A[j * n + i]) > 1e-9 * std::max(scale, 1e-300)) return false;
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int t = 0; t < j; ++t) s -= L[j * n + t] * L[j * n + t];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    L[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int t = 0; t < j; ++t) v -= L[i * n + t] * L[j * n + t];
      L[i * n + j] = v / d;
    }
  }
  (void)worst_asym;
  return true;
}

static bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

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

// ---------------------------------------------------------------------------
// Engine: everything that depends on the model, dimensions and precision.
// ---------------------------------------------------------------------------
class EngineBase {
 public:
  virtual ~EngineBase() { release(); }
  virtual sm_status setup(const sm_problem& pb, hipStream_t stream) = 0;
  virtual sm_status iterate(int k) = 0;
  virtual sm_status result_host(double* mean, double* cov) = 0;
  virtual sm_status result_device(void* mean, void* cov) = 0;

  sm_status track_deltas(double* out) {
    std::vector<unsigned long long> bits(ntracks + 1);
    hipError_t e = hipMemcpyAsync(bits.data(), delta_bits, sizeof(unsigned long long) * (ntracks + 1),
                                  hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "copy of the convergence statistic"));
    for (int i = 0; i <= ntracks; ++i) std::memcpy(&out[i], &bits[i], sizeof(double));
    return SM_OK;
  }

  // Per-launch HIP events (only while profiling).
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
    int64_t positions;
  };

  template <class F>
  void timed(const char* name, int64_t positions, F&& launch) {
    if (!profiling) {
      launch();
      return;
    }
    ProfRec r{name, nullptr, nullptr, positions};
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, stream);
    launch();
    (void)hipEventRecord(r.b, stream);
    prof.push_back(r);
  }

  sm_status profile(int k, sm_kernel_time* out, int cap_out, int* n_out) {
    prof.clear();
    profiling = true;
    sm_status st = iterate(k);
    profiling = false;
    hipError_t e = hipStreamSynchronize(stream);
    std::vector<sm_kernel_time> acc;
    for (ProfRec& r : prof) {
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
      auto it = std::find_if(acc.begin(), acc.end(),
                             [&](const sm_kernel_time& t) { return std::strcmp(t.name, r.name) == 0; });
      if (it == acc.end()) {
        sm_kernel_time t{};
        std::snprintf(t.name, sizeof(t.name), "%s", r.name);
        acc.push_back(t);
        it = acc.end() - 1;
      }
      it->launches += 1;
      it->total_ms += ms;
      it->positions += r.positions;
    }
    prof.clear();
    if (st != SM_OK) return st;
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "profiling events"));
    const int n = std::min<int>(cap_out, int(acc.size()));
    for (int i = 0; i < n; ++i) out[i] = acc[i];
    if (n_out) *n_out = n;
    return SM_OK;
  }

  sm_status fail(sm_status st, const std::string& msg) {
    err = msg;
    return st;
  }

  hipError_t dalloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    if (cap > 0 && int64_t(device_bytes + bytes) > cap) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) {
      allocs.push_back(*p);
      device_bytes += bytes;
    } else {
      *p = nullptr;
    }
    return e;
  }

  void release() {
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
    device_bytes = 0;
  }

  std::string err;
  int64_t S = 0;
  size_t stride = 0;
  int ntracks = 0;
  int n_iter = 0;
  int iters = 0;
  int64_t cap = 0;
  size_t device_bytes = 0;
  hipStream_t stream = nullptr;
  unsigned long long* delta_bits = nullptr;
  std::vector<void*> allocs;
  bool profiling = false;
  std::vector<ProfRec> prof;
};

template <class Model, typename R>
class Engine final : public EngineBase {
 public:
  static constexpr int N = Model::N, P = Model::P;
  static constexpr int kSN = sym_size<N>();
  static constexpr int kTrajW = N + kSN;
  using FOp = FilterOp<N, R>;
  using SOp = SmootherOp<N, R>;
  using LL = LinLayout<N, P>;

  sm_status setup(const sm_problem& pb, hipStream_t st) override {
    stream = st;
    cap = pb.max_device_bytes;
    ntracks = pb.n_tracks;
    n_iter = pb.n_iter;
    lin_ = pb.lin;
    seq_ = pb.scan == SM_SCAN_SEQUENTIAL;
    rule_.alpha = pb.ut_alpha;
    rule_.kappa = pb.ut_kappa;
    // slot map
    slot_off_.resize(ntracks + 1);
    for (int i = 0; i <= ntracks; ++i) slot_off_[i] = pb.offsets[i] + i;
    S = slot_off_[ntracks];
    stride = size_t((S + 63) / 64 * 64);
    std::vector<unsigned char> flags(S, 0);
    std::vector<int> track(S, 0);
    for (int i = 0; i < ntracks; ++i) {
      for (int64_t s = slot_off_[i]; s < slot_off_[i + 1]; ++s) track[s] = i;
      flags[slot_off_[i]] |= kSlotFirst;
      flags[slot_off_[i + 1] - 1] |= kSlotLast;
    }
    // host copies in the compute precision
    std::vector<R> prm(pb.params, pb.params + pb.n_params);
    std::vector<R> Q(pb.Q, pb.Q + N * N), Rm(pb.R, pb.R + P * P);
    std::vector<R> m0(size_t(N) * ntracks), P0(size_t(kSN) * ntracks);
    for (int t = 0; t < ntracks; ++t) {
      for (int i = 0; i < N; ++i) m0[size_t(i) * ntracks + t] = R(pb.m0[size_t(t) * N + i]);
      for (int i = 0; i < N; ++i)
        for (int j = i; j < N; ++j)
          P0[size_t(sym_index<N>(i, j)) * ntracks + t] = R(pb.P0[(size_t(t) * N + i) * N + j]);
    }
    std::vector<R> yslot(size_t(P) * stride, R(0));
    for (int t = 0; t < ntracks; ++t)
      for (int64_t k = 1; k < slot_off_[t + 1] - slot_off_[t]; ++k) {
        const int64_t s = slot_off_[t] + k, row = pb.offsets[t] + k - 1;
        for (int i = 0; i < P; ++i) yslot[size_t(i) * stride + s] = R(pb.y[row * P + i]);
      }
    levels_ = plan_levels(S);
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
    A(&d_traj_[0], sizeof(R) * kTrajW * stride);
    A(&d_traj_[1], sizeof(R) * kTrajW * stride);
    A(&d_lin_, sizeof(R) * LL::kWords * stride);
    A(&d_filt_, sizeof(R) * kTrajW * stride);
    A(reinterpret_cast<void**>(&delta_bits), sizeof(unsigned long long) * (ntracks + 1));
    if (!seq_) {
      // smoothing elements reuse the filtering-element buffer (dead after the prefix scan)
      A(&d_felem_, sizeof(R) * FOp::kElemWords * stride);
      for (size_t l = 0; l + 1 < levels_.size(); ++l) {
        ScanLevel& L = levels_[l];
        A(&L.lane_excl, sizeof(R) * FOp::kElemWords * L.tiles * kScanB);
        A(&L.tile_agg, sizeof(R) * FOp::kElemWords * L.tiles);
        A(&L.tile_carry, sizeof(R) * FOp::kCarryWords * L.tiles);
      }
    }
    if (e != hipSuccess)
      return fail(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE,
                  hip_msg(e, "device allocation") + " (plan needs more than is available or allowed)");
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
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "upload of the problem"));
    const int64_t grid = (S + kSlotBlock - 1) / kSlotBlock;
    SlotArgs a = args(0);
    if (pb.init_mean) {
      // caller trajectory: pack on the device from staging copies
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
        hipLaunchKernelGGL((k_pack<N, R>), dim3(grid), dim3(kSlotBlock), 0, stream, S, stride,
                           static_cast<const R*>(dm), static_cast<const R*>(dc), static_cast<R*>(d_traj_[0]));
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
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "initial trajectory"));
    cur_ = 0;
    return SM_OK;
  }

  SlotArgs args(int cur) const {
    SlotArgs a;
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
    a.felem = d_felem_;
    a.filt = d_filt_;
    a.selem = d_felem_;
    a.traj_out = d_traj_[cur ^ 1];
    a.delta_bits = delta_bits;
    a.rule = rule_;
    return a;
  }

  template <class Op>
  void run_scan(const void* elems, bool reverse, void* out, const char* const (&names)[3]) {
    const size_t lds = sizeof(R) * Op::kElemWords * kScanB;
    const int L = int(levels_.size());
    for (int l = 0; l + 1 < L; ++l) {
      const ScanLevel& lv = levels_[l];
      ScanArgs a{};
      a.elems = l == 0 ? elems : levels_[l - 1].tile_agg;
      a.estride = l == 0 ? stride : size_t(levels_[l - 1].tiles);
      a.m = lv.m;
      a.reverse = (l == 0 && reverse) ? 1 : 0;
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
      a.estride = L == 1 ? stride : size_t(levels_[L - 2].tiles);
      a.m = top.m;
      a.reverse = (L == 1 && reverse) ? 1 : 0;
      a.K = top.K;
      a.out = L == 1 ? out : levels_[L - 2].tile_carry;
      a.ostride = L == 1 ? stride : size_t(levels_[L - 2].tiles);
      timed(names[1], top.m, [&] {
        hipLaunchKernelGGL((k_scan_single<Op, kScanB, R>), dim3(1), dim3(kScanB), lds, stream, a);
      });
    }
    for (int l = L - 2; l >= 0; --l) {
      const ScanLevel& lv = levels_[l];
      ScanArgs a{};
      a.elems = l == 0 ? elems : levels_[l - 1].tile_agg;
      a.estride = l == 0 ? stride : size_t(levels_[l - 1].tiles);
      a.m = lv.m;
      a.reverse = (l == 0 && reverse) ? 1 : 0;
      a.K = lv.K;
      a.lane_excl = lv.lane_excl;
      a.lstride = size_t(lv.tiles) * kScanB;
      a.tile_carry = lv.tile_carry;
      a.cstride = size_t(lv.tiles);
      a.out = l == 0 ? out : levels_[l - 1].tile_carry;
      a.ostride = l == 0 ? stride : size_t(levels_[l - 1].tiles);
      timed(names[2], lv.m, [&] {
        hipLaunchKernelGGL((k_scan_down<Op, kScanB, R>), dim3(lv.tiles), dim3(kScanB), 0, stream, a);
      });
    }
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
    static const char* const kFilterNames[3] = {"scan_up_filter", "scan_top_filter", "scan_down_filter"};
    static const char* const kSmootherNames[3] = {"scan_up_smoother", "scan_top_smoother", "scan_down_smoother"};
    const dim3 grid(unsigned((S + kSlotBlock - 1) / kSlotBlock));
    for (int it = 0; it < k; ++it) {
      const SlotArgs a = args(cur_);
      timed("reset_delta", ntracks + 1, [&] {
        hipLaunchKernelGGL(k_fill_u64, dim3((ntracks + 256) / 256), dim3(256), 0, stream, delta_bits,
                           int64_t(ntracks + 1), 0ull);
      });
      timed("linearize", S, [&] { launch_linearize(a, grid); });
      if (seq_) {
        timed("sequential", S, [&] {
          hipLaunchKernelGGL((k_sequential<N, P, R>), dim3((ntracks + 63) / 64), dim3(64), 0, stream, a,
                             d_slot_off_, ntracks);
        });
      } else {
        timed("filter_elements", S, [&] {
          hipLaunchKernelGGL((k_filter_elements<N, P, R>), grid, dim3(kSlotBlock), 0, stream, a);
        });
        run_scan<FOp>(d_felem_, false, d_filt_, kFilterNames);
        timed("smoother_elements", S, [&] {
          hipLaunchKernelGGL((k_smoother_elements<N, P, R>), grid, dim3(kSlotBlock), 0, stream, a);
        });
        run_scan<SOp>(d_felem_, true, d_traj_[cur_ ^ 1], kSmootherNames);
      }
      timed("delta", S, [&] { hipLaunchKernelGGL((k_delta<N, R>), grid, dim3(kSlotBlock), 0, stream, a); });
      cur_ ^= 1;
      ++iters;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "kernel launch"));
    return SM_OK;
  }

  sm_status result_host(double* mean, double* cov) override {
    std::vector<R> h(size_t(kTrajW) * stride);
    hipError_t e = hipMemcpyAsync(h.data(), d_traj_[cur_], sizeof(R) * h.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "copy of the result"));
    for (int64_t s = 0; s < S; ++s) {
      if (mean)
        for (int i = 0; i < N; ++i) mean[size_t(s) * N + i] = double(h[size_t(i) * stride + s]);
      if (cov)
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j)
            cov[(size_t(s) * N + i) * N + j] = double(h[size_t(N + sym_index<N>(i, j)) * stride + s]);
    }
    return SM_OK;
  }

  sm_status result_device(void* mean, void* cov) override {
    const dim3 grid(unsigned((S + kSlotBlock - 1) / kSlotBlock));
    hipLaunchKernelGGL((k_unpack<N, R>), grid, dim3(kSlotBlock), 0, stream, S, stride,
                       static_cast<const R*>(d_traj_[cur_]), static_cast<R*>(mean), static_cast<R*>(cov));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "result kernel"));
    return SM_OK;
  }

 private:
  int lin_ = 0;
  bool seq_ = false;
  SigmaRule rule_{1.0, 1.0};
  int cur_ = 0;
  std::vector<int64_t> slot_off_;
  std::vector<ScanLevel> levels_;
  void *d_params_ = nullptr, *d_Q_ = nullptr, *d_R_ = nullptr, *d_m0_ = nullptr, *d_P0_ = nullptr;
  unsigned char* d_flags_ = nullptr;
  int* d_track_ = nullptr;
  int64_t* d_slot_off_ = nullptr;
  void *d_y_ = nullptr, *d_traj_[2] = {nullptr, nullptr}, *d_lin_ = nullptr, *d_filt_ = nullptr;
  void* d_felem_ = nullptr;
};

// Compiled (model, nx, ny) combinations.
template <typename R>
static EngineBase* make_engine_t(int model, int nx, int ny) {
  if (model == SM_MODEL_CT_BEARINGS) {
    if (nx == 5 && ny == 2) return new Engine<CtBearings<5, 2, R>, R>();
  } else if (model == SM_MODEL_LINEAR) {
    if (nx == 1 && ny == 1) return new Engine<LinearModel<1, 1, R>, R>();
    if (nx == 3 && ny == 2) return new Engine<LinearModel<3, 2, R>, R>();
    if (nx == 5 && ny == 2) return new Engine<LinearModel<5, 2, R>, R>();
  }
  return nullptr;
}

static bool supported(int model, int nx, int ny) {
  if (model == SM_MODEL_CT_BEARINGS) return nx == 5 && ny == 2;
  if (model == SM_MODEL_LINEAR) return (nx == 1 && ny == 1) || (nx == 3 && ny == 2) || (nx == 5 && ny == 2);
  return false;
}

static std::string validate(const sm_problem* pb) {
  if (!pb) return "problem is NULL";
  if (pb->model != SM_MODEL_LINEAR && pb->model != SM_MODEL_CT_BEARINGS) return "unknown model";
  if (!supported(pb->model, pb->nx, pb->ny))
    return "unsupported (model, nx, ny) = (" + std::to_string(pb->model) + ", " + std::to_string(pb->nx) + ", " +
           std::to_string(pb->ny) + ")";
  const int n = pb->nx, p = pb->ny;
  if (pb->n_tracks < 1) return "n_tracks must be >= 1";
  if (!pb->offsets) return "offsets is NULL";
  if (pb->offsets[0] != 0) return "offsets[0] must be 0";
  for (int i = 0; i < pb->n_tracks; ++i)
    if (pb->offsets[i + 1] <= pb->offsets[i]) return "every track needs T >= 1 (offsets must increase)";
  const int64_t nmeas = pb->offsets[pb->n_tracks];
  if (nmeas + pb->n_tracks > int64_t(INT32_MAX)) return "too many slots";
  if (!pb->params) return "params is NULL";
  if (pb->model == SM_MODEL_LINEAR) {
    if (pb->n_params != n * n + n + p * n + p) return "LINEAR model needs nx*nx + nx + ny*nx + ny params";
  } else {
    if (pb->n_params != 1 + 3 * p) return "CT_BEARINGS model needs 1 + 3*ny params";
    if (!(pb->params[0] > 0.0) || !std::isfinite(pb->params[0])) return "dt must be positive and finite";
    for (int s = 0; s < p; ++s) {
      const double t = pb->params[3 + 3 * s];
      if (!(t >= 0.0) || t >= n / 5 || t != std::floor(t)) return "sensor target index out of range";
    }
  }
  if (!all_finite(pb->params, size_t(pb->n_params))) return "params must be finite";
  if (!pb->Q || !pb->R || !pb->m0 || !pb->P0 || !pb->y) return "Q, R, m0, P0 and y must not be NULL";
  if (!host_spd(pb->Q, n)) return "Q must be symmetric positive definite";
  if (!host_spd(pb->R, p)) return "R must be symmetric positive definite";
  if (!all_finite(pb->m0, size_t(pb->n_tracks) * n)) return "m0 must be finite";
  for (int t = 0; t < pb->n_tracks; ++t)
    if (!host_spd(pb->P0 + size_t(t) * n * n, n)) return "P0 of track " + std::to_string(t) + " must be SPD";
  if (!all_finite(pb->y, size_t(nmeas) * p)) return "y must be finite";
  if (pb->n_iter < 0) return "n_iter must be >= 0";
  if (pb->lin < SM_LIN_TAYLOR || pb->lin > SM_LIN_UNSCENTED) return "unknown linearisation";
  if (pb->lin == SM_LIN_UNSCENTED) {
    const double lam = pb->ut_alpha * pb->ut_alpha * (n + pb->ut_kappa) - n;
    if (!(n + lam > 0.0)) return "unscented parameters give n + lambda <= 0";
  }
  if (pb->precision != SM_FP64 && pb->precision != SM_FP32) return "unknown precision";
  if (pb->scan != SM_SCAN_PARALLEL && pb->scan != SM_SCAN_SEQUENTIAL) return "unknown scan mode";
  if (pb->max_device_bytes < 0) return "max_device_bytes must be >= 0";
  const int64_t S = nmeas + pb->n_tracks;
  if (pb->init_cov && !pb->init_mean) return "init_cov given without init_mean";
  if (pb->init_mean && !all_finite(pb->init_mean, size_t(S) * n)) return "init_mean must be finite";
  if (pb->init_cov)
    for (int64_t s = 0; s < S; ++s)
      if (!host_spd(pb->init_cov + size_t(s) * n * n, n)) return "init_cov must be SPD at every slot";
  return std::string();
}

}  // namespace pks

struct smoother {
  std::unique_ptr<pks::EngineBase> eng;
  std::string err;
};

using pks::g_init_error;

extern "C" {

void smoother_problem_defaults(sm_problem* pb) {
  if (!pb) return;
  std::memset(pb, 0, sizeof(*pb));
  pb->n_tracks = 1;
  pb->n_iter = 10;
  pb->lin = SM_LIN_TAYLOR;
  pb->ut_alpha = 1.0;
  pb->ut_beta = 0.0;
  pb->ut_kappa = 1.0;
  pb->precision = SM_FP64;
  pb->scan = SM_SCAN_PARALLEL;
}

sm_status smoother_init(const sm_problem* pb, void* hip_stream, smoother_t* out) {
  if (out) *out = nullptr;
  try {
    if (!out) {
      g_init_error = "out is NULL";
      return SM_EINVAL;
    }
    const std::string msg = pks::validate(pb);
    if (!msg.empty()) {
      g_init_error = msg;
      return SM_EINVAL;
    }
    std::unique_ptr<pks::EngineBase> eng(pb->precision == SM_FP64
                                             ? pks::make_engine_t<double>(pb->model, pb->nx, pb->ny)
                                             : pks::make_engine_t<float>(pb->model, pb->nx, pb->ny));
    if (!eng) {
      g_init_error = "no kernel for this configuration";
      return SM_EINVAL;
    }
    const sm_status st = eng->setup(*pb, static_cast<hipStream_t>(hip_stream));
    if (st != SM_OK) {
      g_init_error = eng->err;
      return st;
    }
    smoother* h = new smoother();
    h->eng = std::move(eng);
    *out = h;
    g_init_error.clear();
    return SM_OK;
  } catch (const std::bad_alloc&) {
    g_init_error = "host allocation failed";
    return SM_ENOMEM;
  } catch (...) {
    g_init_error = "unexpected host exception";
    return SM_EDEVICE;
  }
}

sm_status smoother_iterate(smoother_t h, int32_t k, double* max_delta_out, int32_t* iters_done_out) {
  if (!h || !h->eng) return SM_ESTATE;
  try {
    pks::EngineBase& e = *h->eng;
    const int todo = k > 0 ? k : std::max(0, e.n_iter - e.iters);
    sm_status st = e.iterate(todo);
    if (st != SM_OK) {
      h->err = e.err;
      return st;
    }
    if (iters_done_out) *iters_done_out = e.iters;
    if (max_delta_out) {
      std::vector<double> d(e.ntracks + 1);
      st = e.track_deltas(d.data());
      if (st != SM_OK) {
        h->err = e.err;
        return st;
      }
      *max_delta_out = d[e.ntracks];
      if (!std::isfinite(d[e.ntracks])) {
        h->err = "non-finite iterate";
        return SM_ENUMERIC;
      }
    }
    return SM_OK;
  } catch (...) {
    h->err = "unexpected host exception";
    return SM_EDEVICE;
  }
}

sm_status smoother_result(smoother_t h, double* mean, double* cov) {
  if (!h || !h->eng) return SM_ESTATE;
  try {
    const sm_status st = h->eng->result_host(mean, cov);
    if (st != SM_OK) h->err = h->eng->err;
    return st;
  } catch (...) {
    h->err = "unexpected host exception";
    return SM_EDEVICE;
  }
}

sm_status smoother_result_device(smoother_t h, void* d_mean, void* d_cov) {
  if (!h || !h->eng) return SM_ESTATE;
  const sm_status st = h->eng->result_device(d_mean, d_cov);
  if (st != SM_OK) h->err = h->eng->err;
  return st;
}

sm_status smoother_track_deltas(smoother_t h, double* deltas) {
  if (!h || !h->eng) return SM_ESTATE;
  if (!deltas) {
    h->err = "deltas is NULL";
    return SM_EINVAL;
  }
  try {
    std::vector<double> d(h->eng->ntracks + 1);
    const sm_status st = h->eng->track_deltas(d.data());
    if (st != SM_OK) {
      h->err = h->eng->err;
      return st;
    }
    std::memcpy(deltas, d.data(), sizeof(double) * h->eng->ntracks);
    return SM_OK;
  } catch (...) {
    h->err = "unexpected host exception";
    return SM_EDEVICE;
  }
}

sm_status smoother_profile(smoother_t h, int32_t k, sm_kernel_time* out, int32_t cap, int32_t* n_out) {
  if (!h || !h->eng) return SM_ESTATE;
  if (!out || cap < 1 || k < 1) {
    h->err = "profile needs k >= 1 and an output array";
    return SM_EINVAL;
  }
  try {
    const sm_status st = h->eng->profile(k, out, cap, n_out);
    if (st != SM_OK) h->err = h->eng->err;
    return st;
  } catch (...) {
    h->err = "unexpected host exception";
    return SM_EDEVICE;
  }
}

sm_status smoother_info(smoother_t h, int64_t* n_slots, int32_t* n_tracks, int64_t* device_bytes) {
  if (!h || !h->eng) return SM_ESTATE;
  if (n_slots) *n_slots = h->eng->S;
  if (n_tracks) *n_tracks = h->eng->ntracks;
  if (device_bytes) *device_bytes = int64_t(h->eng->device_bytes);
  return SM_OK;
}

const char* smoother_last_error(smoother_t h) {
  if (!h) return g_init_error.c_str();
  return h->err.c_str();
}

void smoother_destroy(smoother_t h) {
  if (!h) return;
  if (h->eng) (void)hipStreamSynchronize(h->eng->stream);
  delete h;
}

const char* smoother_version(void) { return "pks-0.1 gfx950"; }

}  // extern "C"
