// C ABI of the parallel iterated smoother (include/smoother.h): host-side
// validation of the problem, handle lifetime and error reporting.  The device
// memory plan and the kernel sequence live in the engines (engine.hpp), one
// translation unit per model and precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "smoother.h"
#include "block_engine.hpp"
#include "engine_base.hpp"

namespace pks {

static thread_local std::string g_init_error;

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

// Symmetric positive semi-definite: a Cholesky factorisation in which a pivot
// at or below 1e-12 times the largest diagonal entry is a direction without
// variance.  Its remaining column must then vanish up to what such a pivot
// allows (at most sqrt(1e-12) times the largest diagonal entry, with a
// margin): [[0, 1], [1, 1]] is rejected.
static bool host_psd(const double* A, int n) {
  std::vector<double> L(size_t(n) * n, 0.0);
  double scale = 0.0, dmax = 0.0;
  for (int i = 0; i < n * n; ++i) {
    if (!std::isfinite(A[i])) return false;
    scale = std::max(scale, std::fabs(A[i]));
  }
  for (int i = 0; i < n; ++i) {
    dmax = std::max(dmax, A[i * n + i]);
    for (int j = i + 1; j < n; ++j)
      if (std::fabs(A[i * n + j] - A[j * n + i]) > 1e-9 * std::max(scale, 1e-300)) return false;
  }
  const double tiny = 1e-12 * dmax;
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int t = 0; t < j; ++t) s -= L[j * n + t] * L[j * n + t];
    if (s < -tiny) return false;
    const bool live = s > tiny;
    const double d = live ? std::sqrt(s) : 0.0;
    L[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int t = 0; t < j; ++t) v -= L[i * n + t] * L[j * n + t];
      if (!live && std::fabs(v) > 2e-6 * dmax) return false;
      L[i * n + j] = live ? v / d : 0.0;
    }
  }
  return true;
}

static bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static EngineBase* make_dense_engine(int model, int precision, int nx, int ny) {
  if (model == SM_MODEL_CT_BEARINGS)
    return precision == SM_FP64 ? make_engine_ct_f64(nx, ny) : make_engine_ct_f32(nx, ny);
  if (model == SM_MODEL_LINEAR)
    return precision == SM_FP64 ? make_engine_linear_f64(nx, ny) : make_engine_linear_f32(nx, ny);
  return nullptr;
}

constexpr int kMaxTargets = 16;   // coordinated-turn blocks in one stacked state

static bool stacked(int model, int nx) { return model == SM_MODEL_CT_BEARINGS && nx > 5 && nx % 5 == 0; }

// Stacked targets: the Taylor linearisation runs each target as its own block;
// sigma-point rules couple the targets and run on the wavefront-cooperative
// engine of the full state.
static EngineBase* make_engine(int model, int precision, int nx, int ny, int lin) {
  if (stacked(model, nx)) {
    if (lin != SM_LIN_TAYLOR)
      return precision == SM_FP64 ? make_engine_dense_ct_f64(nx, ny) : make_engine_dense_ct_f32(nx, ny);
    BlockEngine* e = new BlockEngine(&make_dense_engine);
    e->set_precision_word(precision == SM_FP64 ? sizeof(double) : sizeof(float));
    return e;
  }
  return make_dense_engine(model, precision, nx, ny);
}

static bool supported(int model, int nx, int ny, int lin, int precision) {
  if (model == SM_MODEL_CT_BEARINGS) {
    if (nx == 5) return ny == 2;
    if (!stacked(model, nx)) return false;
    // sigma points: the compiled full-state engine (four targets, eight sensors)
    if (lin != SM_LIN_TAYLOR) return nx == 20 && ny == 8;
    // Taylor: two sensors per target, blocks run on the (5, 2) kernels
    return nx / 5 <= kMaxTargets && ny == 2 * (nx / 5);
  }
  if (model == SM_MODEL_LINEAR) return (nx == 1 && ny == 1) || (nx == 3 && ny == 2) || (nx == 5 && ny == 2);
  return false;
}

// Entries of the symmetric n x n matrix A between different blocks (block(i)
// gives the block of index i) are zero up to rounding: |A_ij| <= 1e-12
// sqrt(A_ii A_jj).  Such entries are dropped by the block decomposition.
template <class F>
static bool block_diagonal(const double* A, int n, F block) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (block(i) != block(j) &&
          !(std::fabs(A[i * n + j]) <= 1e-12 * std::sqrt(std::fabs(A[i * n + i] * A[j * n + j]))))
        return false;
  return true;
}

static std::string validate(const sm_problem* pb) {
  if (!pb) return "problem is NULL";
  if (pb->model != SM_MODEL_LINEAR && pb->model != SM_MODEL_CT_BEARINGS) return "unknown model";
  if (!supported(pb->model, pb->nx, pb->ny, pb->lin, pb->precision))
    return "unsupported (model, nx, ny, linearisation, precision) = (" + std::to_string(pb->model) + ", " +
           std::to_string(pb->nx) + ", " + std::to_string(pb->ny) + ", " + std::to_string(pb->lin) + ", " +
           std::to_string(pb->precision) + ")";
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
  if (pb->form == SM_FORM_SQRT ? !host_psd(pb->Q, n) : !host_spd(pb->Q, n))
    return pb->form == SM_FORM_SQRT ? "Q must be symmetric positive semi-definite"
                                    : "Q must be symmetric positive definite (the square-root form takes a "
                                      "positive semi-definite Q)";
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
  if (pb->tile_lanes != 0 && pb->tile_lanes != 64 && pb->tile_lanes != 256) return "tile_lanes must be 0, 64 or 256";
  if (pb->lane_slots < 0 || pb->lane_slots > 32) return "lane_slots must be in 0..32";
  if (pb->use_graph != 0 && pb->use_graph != 1) return "use_graph must be 0 or 1";
  if (!(pb->lm_lambda >= 0.0) || !std::isfinite(pb->lm_lambda)) return "lm_lambda must be finite and >= 0";
  if (pb->form != SM_FORM_COVARIANCE && pb->form != SM_FORM_SQRT) return "unknown element form";
  if (pb->freeze_converged != 0 && pb->freeze_converged != 1) return "freeze_converged must be 0 or 1";
  if (pb->form == SM_FORM_SQRT) {
    if (pb->scan != SM_SCAN_PARALLEL) return "the square-root form runs on the parallel scan";
    if (pb->lm_lambda != 0.0) return "the square-root form runs without damping (lm_lambda must be 0)";
    if (stacked(pb->model, n) && pb->lin != SM_LIN_TAYLOR)
      return "the square-root form is not built for the full-state (nx = 20 sigma-point) engine";
  }
  const int64_t S = nmeas + pb->n_tracks;
  if (pb->init_cov && !pb->init_mean) return "init_cov given without init_mean";
  if (pb->init_mean && !all_finite(pb->init_mean, size_t(S) * n)) return "init_mean must be finite";
  if (pb->init_cov)
    for (int64_t s = 0; s < S; ++s)
      if (!host_spd(pb->init_cov + size_t(s) * n * n, n)) return "init_cov must be SPD at every slot";
  if (stacked(pb->model, n) && pb->lin == SM_LIN_TAYLOR) {
    // the targets must not interact for the block decomposition to be exact
    const int k = n / 5;
    std::vector<int> per(k, 0);
    for (int s = 0; s < p; ++s) per[int(pb->params[3 + 3 * s])] += 1;
    for (int b = 0; b < k; ++b)
      if (per[b] != 2) return "stacked targets: every target needs exactly two sensors";
    auto sblk = [](int i) { return i / 5; };
    auto mblk = [&](int s) { return int(pb->params[3 + 3 * s]); };
    if (!block_diagonal(pb->Q, n, sblk)) return "stacked targets: Q must be block-diagonal";
    if (!block_diagonal(pb->R, p, mblk)) return "stacked targets: R must not couple sensors of different targets";
    for (int t = 0; t < pb->n_tracks; ++t)
      if (!block_diagonal(pb->P0 + size_t(t) * n * n, n, sblk)) return "stacked targets: P0 must be block-diagonal";
    if (pb->init_cov)
      for (int64_t s = 0; s < S; ++s)
        if (!block_diagonal(pb->init_cov + size_t(s) * n * n, n, sblk))
          return "stacked targets: init_cov must be block-diagonal";
  }
  return std::string();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (smoother_solve_static): one
// array per GPU, loaded with the code object and held until the process
// ends.  In host code `scratch` names a host-side stand-in only; the device
// address of each GPU's copy comes from hipGetSymbolAddress with that device
// current, and only that address is handed to the engine and its kernels.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int64_t kStaticMaxSlots = 36864;   // sum over tracks of T_i + 1
constexpr int kStaticMaxTracks = 1024;
constexpr int kStaticMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kStaticMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device.
static hipError_t static_scratch(void** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kStaticMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace pks

struct smoother {
  std::unique_ptr<pks::EngineBase> eng;
  std::string err;
  int nx = 0;
  int precision = SM_FP64;
  bool blocks = false;    // stacked targets run as separate blocks
  bool q_definite = true; // Q positive definite (the MAP objective needs Q^-1)
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
  pb->use_graph = 1;
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
    std::unique_ptr<pks::EngineBase> eng(pks::make_engine(pb->model, pb->precision, pb->nx, pb->ny, pb->lin));
    if (!eng) {
      g_init_error = "no kernel for this configuration";
      return SM_EINVAL;
    }
    const sm_status st = eng->setup(*pb, static_cast<hipStream_t>(hip_stream));
    if (st != SM_OK) {
      g_init_error = eng->err;
      return st;
    }
    eng->freeze_converged = pb->freeze_converged != 0;
    smoother* h = new smoother();
    h->eng = std::move(eng);
    h->nx = pb->nx;
    h->precision = pb->precision;
    h->q_definite = pks::host_spd(pb->Q, pb->nx);
    h->blocks = pks::stacked(pb->model, pb->nx) && pb->lin == SM_LIN_TAYLOR;
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

sm_status smoother_autotune(const sm_problem* pb, void* hip_stream, int32_t iters, int32_t* tile_lanes,
                            int32_t* lane_slots, double* ms_per_iter) {
  try {
    if (!pb || !tile_lanes || !lane_slots || iters < 1) {
      g_init_error = "autotune needs a problem, output pointers and iters >= 1";
      return SM_EINVAL;
    }
    const std::string msg = pks::validate(pb);
    if (!msg.empty()) {
      g_init_error = msg;
      return SM_EINVAL;
    }
    if (pb->scan != SM_SCAN_PARALLEL) {
      g_init_error = "autotune applies to the parallel scan";
      return SM_EINVAL;
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t he = hipEventCreate(&a);
    if (he == hipSuccess) he = hipEventCreate(&b);
    if (he != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      g_init_error = pks::hip_msg(he, "autotune events");
      return SM_EDEVICE;
    }
    double best = -1.0;
    int best_b = 0, best_k = 0;
    sm_status last = SM_OK;
    std::string last_err;
    // schedules as the engines run them: the square-root form and the
    // full-state engine fix the tile width, so two candidates can be one
    std::vector<std::pair<int, int>> timed;
    for (const int lanes : {64, 256}) {
      for (const int slots : {1, 2, 4, 8, 16}) {
        sm_problem q = *pb;
        q.tile_lanes = lanes;
        q.lane_slots = slots;
        std::unique_ptr<pks::EngineBase> eng(pks::make_engine(q.model, q.precision, q.nx, q.ny, q.lin));
        if (!eng) {
          last = SM_EINVAL;
          last_err = "no kernel for this configuration";
          continue;
        }
        q.n_iter = 3 * iters + 1;
        sm_status st = eng->setup(q, stream);
        if (st == SM_OK) {
          const std::pair<int, int> actual{eng->sched_lanes, eng->sched_slots};
          if (std::find(timed.begin(), timed.end(), actual) != timed.end()) {
            (void)hipStreamSynchronize(stream);   // setup's work done before the handle is released
            continue;
          }
          timed.push_back(actual);
          st = eng->iterate(1);                                 // warm-up (and graph capture)
        }
        // best of three timed rounds of `iters` iterations (candidates a few
        // percent apart would otherwise swap places from run to run)
        float ms = 0.f;
        for (int round = 0; round < 3 && st == SM_OK; ++round) {
          float t = 0.f;
          he = hipEventRecord(a, stream);
          if (he == hipSuccess) st = eng->iterate(iters);
          if (he == hipSuccess && st == SM_OK) he = hipEventRecord(b, stream);
          if (he == hipSuccess && st == SM_OK) he = hipEventSynchronize(b);
          if (he == hipSuccess && st == SM_OK) he = hipEventElapsedTime(&t, a, b);
          if (he != hipSuccess) {
            st = SM_EDEVICE;
            eng->err = pks::hip_msg(he, "autotune timing");
          }
          if (round == 0 || t < ms) ms = t;
        }
        (void)hipStreamSynchronize(stream);   // nothing of this candidate in flight when it is released
        if (st != SM_OK) {            // e.g. a schedule that does not fit the memory cap
          last = st;
          last_err = eng->err;
          continue;
        }
        const double per = double(ms) / iters;
        if (best < 0.0 || per < best) {
          best = per;
          best_b = eng->sched_lanes;
          best_k = eng->sched_slots;
        }
      }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (best < 0.0) {
      g_init_error = "no schedule could run: " + last_err;
      return last == SM_OK ? SM_EDEVICE : last;
    }
    *tile_lanes = best_b;
    *lane_slots = best_k;
    if (ms_per_iter) *ms_per_iter = best;
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

}  // extern "C"

namespace {

// Schedules found by smoother_autotune_cached, per process.  The time of a
// schedule depends on the problem's shape, not on its values: the key holds
// the device, every field that selects kernels, sizes the plan or changes how
// an iteration is launched (graph replay or not), and an FNV-1a hash of the
// track offsets.
struct TuneRec {
  int32_t lanes, slots;
  double ms;
};
std::mutex g_tune_mutex;
std::vector<std::pair<std::string, TuneRec>> g_tune_cache;

std::string tune_key(const sm_problem* pb, int32_t iters) {
  int dev = -1;
  (void)hipGetDevice(&dev);
  uint64_t h = 1469598103934665603ull;
  const unsigned char* o = reinterpret_cast<const unsigned char*>(pb->offsets);
  for (size_t i = 0; i < sizeof(int64_t) * size_t(pb->n_tracks + 1); ++i) h = (h ^ o[i]) * 1099511628211ull;
  char buf[256];
  std::snprintf(buf, sizeof(buf), "d%d m%d n%d p%d t%d l%d pr%d f%d z%d lm%d g%d it%d cap%lld o%016llx", dev,
                pb->model, pb->nx, pb->ny, pb->n_tracks, pb->lin, pb->precision, pb->form, pb->freeze_converged,
                pb->lm_lambda != 0.0 ? 1 : 0, pb->use_graph != 0 ? 1 : 0, iters,
                static_cast<long long>(pb->max_device_bytes), static_cast<unsigned long long>(h));
  return buf;
}

}  // namespace

extern "C" {

sm_status smoother_autotune_cached(const sm_problem* pb, void* hip_stream, int32_t iters, int32_t* tile_lanes,
                                   int32_t* lane_slots, double* ms_per_iter, int32_t* from_cache) {
  try {
    if (!pb || !tile_lanes || !lane_slots || iters < 1) {
      g_init_error = "autotune needs a problem, output pointers and iters >= 1";
      return SM_EINVAL;
    }
    const std::string msg = pks::validate(pb);
    if (!msg.empty()) {
      g_init_error = msg;
      return SM_EINVAL;
    }
    const std::string key = tune_key(pb, iters);
    {
      std::lock_guard<std::mutex> lock(g_tune_mutex);
      for (const auto& e : g_tune_cache)
        if (e.first == key) {
          *tile_lanes = e.second.lanes;
          *lane_slots = e.second.slots;
          if (ms_per_iter) *ms_per_iter = e.second.ms;
          if (from_cache) *from_cache = 1;
          g_init_error.clear();
          return SM_OK;
        }
    }
    double ms = 0.0;
    const sm_status st = smoother_autotune(pb, hip_stream, iters, tile_lanes, lane_slots, &ms);
    if (st != SM_OK) return st;
    {
      std::lock_guard<std::mutex> lock(g_tune_mutex);
      g_tune_cache.push_back({key, TuneRec{*tile_lanes, *lane_slots, ms}});
    }
    if (ms_per_iter) *ms_per_iter = ms;
    if (from_cache) *from_cache = 0;
    return SM_OK;
  } catch (const std::bad_alloc&) {
    g_init_error = "host allocation failed";
    return SM_ENOMEM;
  } catch (...) {
    g_init_error = "unexpected host exception";
    return SM_EDEVICE;
  }
}

void smoother_autotune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_tune_cache.clear();
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

sm_status smoother_iterate_until(smoother_t h, double tol, int32_t max_iter, int32_t* iters_run,
                                 int32_t* track_iters) {
  if (!h || !h->eng) return SM_ESTATE;
  if (!(tol > 0.0) || max_iter < 1) {
    h->err = "iterate_until needs tol > 0 and max_iter >= 1";
    return SM_EINVAL;
  }
  try {
    pks::EngineBase& e = *h->eng;
    std::vector<int32_t> first(e.ntracks);
    int run = 0;
    const sm_status st = e.iterate_until(tol, max_iter, &run, first.data(), e.freeze_converged);
    if (iters_run) *iters_run = run;
    if (track_iters) std::memcpy(track_iters, first.data(), sizeof(int32_t) * e.ntracks);
    if (st != SM_OK) h->err = e.err;
    return st;
  } catch (...) {
    h->err = "unexpected host exception";
    return SM_EDEVICE;
  }
}

sm_status smoother_filter(smoother_t h, double* filt_mean, double* filt_cov, double* track_loglik) {
  if (!h || !h->eng) return SM_ESTATE;
  try {
    const sm_status st = h->eng->filter(filt_mean, filt_cov, track_loglik);
    if (st != SM_OK) h->err = h->eng->err;
    return st;
  } catch (...) {
    h->err = "unexpected host exception";
    return SM_EDEVICE;
  }
}

sm_status smoother_objective(smoother_t h, double* track_cost) {
  if (!h || !h->eng) return SM_ESTATE;
  if (!track_cost) {
    h->err = "track_cost is NULL";
    return SM_EINVAL;
  }
  if (!h->q_definite) {
    h->err = "the MAP objective weighs the process residuals by Q^-1: it needs a positive definite Q";
    return SM_EINVAL;
  }
  try {
    const sm_status st = h->eng->objective(track_cost);
    if (st != SM_OK) h->err = h->eng->err;
    return st;
  } catch (...) {
    h->err = "unexpected host exception";
    return SM_EDEVICE;
  }
}

sm_status smoother_iterate_lm(smoother_t h, double lambda0, double nu, double tol, int32_t max_iter,
                              int32_t* iters_run, int32_t* track_iters, double* track_cost) {
  if (!h || !h->eng) return SM_ESTATE;
  if (!(lambda0 > 0.0) || !std::isfinite(lambda0) || !(nu > 1.0) || !std::isfinite(nu) || !(tol > 0.0) ||
      max_iter < 1) {
    h->err = "iterate_lm needs finite lambda0 > 0, finite nu > 1, tol > 0 and max_iter >= 1";
    return SM_EINVAL;
  }
  try {
    pks::EngineBase& e = *h->eng;
    std::vector<int32_t> first(e.ntracks);
    std::vector<double> cost(e.ntracks);
    int run = 0;
    // a kept step may raise the objective by its rounding level at most
    const double rtol = h->precision == SM_FP64 ? 1e-12 : 1e-6;
    const sm_status st = e.iterate_lm(lambda0, nu, tol, max_iter, rtol, &run, first.data(), cost.data());
    if (iters_run) *iters_run = run;
    if (track_iters) std::memcpy(track_iters, first.data(), sizeof(int32_t) * e.ntracks);
    if (track_cost) std::memcpy(track_cost, cost.data(), sizeof(double) * e.ntracks);
    if (st != SM_OK) h->err = e.err;
    return st;
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

sm_status smoother_set_trajectory_device(smoother_t h, const void* d_mean, const void* d_cov,
                                         const double* cov_const) {
  if (!h || !h->eng) return SM_ESTATE;
  if (!d_mean) {
    h->err = "d_mean is NULL";
    return SM_EINVAL;
  }
  if (d_cov && cov_const) {
    h->err = "give d_cov or cov_const, not both";
    return SM_EINVAL;
  }
  if (cov_const) {
    const int n = h->nx;
    for (int i = 0; i < n * n; ++i)
      if (!std::isfinite(cov_const[i])) {
        h->err = "cov_const must be finite";
        return SM_EINVAL;
      }
    if (!pks::host_spd(cov_const, n)) {
      h->err = "cov_const must be symmetric positive definite";
      return SM_EINVAL;
    }
    if (h->blocks && !pks::block_diagonal(cov_const, n, [](int i) { return i / 5; })) {
      h->err = "stacked targets: cov_const must be block-diagonal";
      return SM_EINVAL;
    }
  }
  try {
    const sm_status st = h->eng->set_trajectory_device(d_mean, d_cov, cov_const);
    if (st != SM_OK) h->err = h->eng->err;
    return st;
  } catch (...) {
    h->err = "unexpected host exception";
    return SM_EDEVICE;
  }
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
  return smoother_profile_repeat(h, k, 1, out, cap, n_out);
}

sm_status smoother_profile_repeat(smoother_t h, int32_t k, int32_t repeat, sm_kernel_time* out, int32_t cap,
                                  int32_t* n_out) {
  if (!h || !h->eng) return SM_ESTATE;
  if (!out || cap < 1 || k < 1 || repeat < 1 || repeat > 64) {
    h->err = "profile needs k >= 1, 1 <= repeat <= 64 and an output array";
    return SM_EINVAL;
  }
  try {
    const sm_status st = h->eng->profile(k, repeat, out, cap, n_out);
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

sm_status smoother_schedule(smoother_t h, int32_t* tile_lanes, int32_t* lane_slots, int64_t* tiles) {
  if (!h || !h->eng) return SM_ESTATE;
  if (tile_lanes) *tile_lanes = h->eng->sched_lanes;
  if (lane_slots) *lane_slots = h->eng->sched_slots;
  if (tiles) *tiles = h->eng->sched_tiles;
  return SM_OK;
}

sm_status smoother_solve_static(const sm_problem* pb, void* hip_stream, void* d_mean, void* d_cov,
                                double* max_delta_out) {
  try {
    const std::string msg = pks::validate(pb);
    if (!msg.empty()) {
      g_init_error = msg;
      return SM_EINVAL;
    }
    if (!d_mean || !d_cov) {
      g_init_error = "d_mean and d_cov must not be NULL";
      return SM_EINVAL;
    }
    if (pb->nx != 5 && !(pb->model == SM_MODEL_LINEAR && pb->nx < 5)) {
      g_init_error = "the static entry point runs the single-block engines only (nx <= 5)";
      return SM_EINVAL;
    }
    if (pb->init_mean || pb->init_cov) {
      g_init_error = "the static entry point starts from the prior broadcast (init_mean and init_cov must be NULL)";
      return SM_EINVAL;
    }
    if (pb->lane_slots > 1) {
      g_init_error = "the static entry point runs one slot per lane (lane_slots must be 0 or 1)";
      return SM_EINVAL;
    }
    const int64_t S = pb->offsets[pb->n_tracks] + pb->n_tracks;
    if (S > pks::kStaticMaxSlots || pb->n_tracks > pks::kStaticMaxTracks) {
      g_init_error = "problem exceeds the static scratch: " + std::to_string(S) + " slots and " +
                     std::to_string(pb->n_tracks) + " tracks given, at most " +
                     std::to_string(pks::kStaticMaxSlots) + " slots (sum of T_i + 1) and " +
                     std::to_string(pks::kStaticMaxTracks) + " tracks";
      return SM_EINVAL;
    }
    void* base = nullptr;
    hipError_t he = pks::static_scratch(&base);
    if (he != hipSuccess) {
      g_init_error = pks::hip_msg(he, "address of the static scratch");
      return SM_EDEVICE;
    }
    std::unique_ptr<pks::EngineBase> eng(pks::make_engine(pb->model, pb->precision, pb->nx, pb->ny, pb->lin));
    if (!eng) {
      g_init_error = "no kernel for this configuration";
      return SM_EINVAL;
    }
    eng->use_arena(base, pks::kStaticScratchBytes);
    sm_problem q = *pb;
    q.use_graph = 0;           // eager launches: a graph would be instantiated (and allocate)
    q.lane_slots = 1;
    q.max_device_bytes = 0;
    sm_status st = eng->setup(q, static_cast<hipStream_t>(hip_stream));
    if (st == SM_OK) st = eng->iterate(q.n_iter);
    if (st == SM_OK) st = eng->result_device(d_mean, d_cov);
    double delta = 0.0;
    if (st == SM_OK && max_delta_out) {
      std::vector<double> d(eng->ntracks + 1);
      st = eng->track_deltas(d.data());
      delta = d[eng->ntracks];
    }
    if (st == SM_OK) {
      he = hipStreamSynchronize(eng->stream);
      if (he != hipSuccess) {
        eng->err = pks::hip_msg(he, "static solve");
        st = SM_EDEVICE;
      }
    }
    if (st != SM_OK) {
      (void)hipStreamSynchronize(eng->stream);
      g_init_error = eng->err;
      return st;
    }
    if (max_delta_out) {
      *max_delta_out = delta;
      if (!std::isfinite(delta)) {
        g_init_error = "non-finite iterate";
        return SM_ENUMERIC;
      }
    }
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
