// Host-side engine interface shared by the C ABI and the per-model
// translation units that instantiate the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "smoother.h"

namespace pks {

inline std::string hip_msg(hipError_t e, const char* what) {
  return std::string(what) + ": " + hipGetErrorString(e);
}

// W = L^-1 for A = L L^T (n x n, row-major, lower triangular), so that
// r^T A^-1 r = |W r|^2.  Returns false if A is not positive definite.
inline bool whitening(const double* A, int n, double* W) {
  std::vector<double> L(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int t = 0; t < j; ++t) d -= L[j * n + t] * L[j * n + t];
    if (!(d > 0.0)) return false;
    L[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int t = 0; t < j; ++t) v -= L[i * n + t] * L[j * n + t];
      L[i * n + j] = v / L[j * n + j];
    }
  }
  // columns of W solve L w = e_c by forward substitution
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double v = i == c ? 1.0 : 0.0;
      for (int t = c; t < i; ++t) v -= L[i * n + t] * W[t * n + c];
      W[i * n + c] = i < c ? 0.0 : v / L[i * n + i];
    }
  return true;
}

constexpr double kLmLambdaMax = 1e16;   // cap of the damping schedule

// Everything that depends on the model, dimensions and precision sits behind this interface.
class EngineBase {
 public:
  virtual ~EngineBase() { release(); }
  virtual sm_status setup(const sm_problem& pb, hipStream_t stream) = 0;
  virtual sm_status iterate(int k) = 0;
  virtual sm_status result_host(double* mean, double* cov) = 0;
  virtual sm_status result_device(void* mean, void* cov) = 0;
  virtual sm_status set_trajectory_device(const void* mean, const void* cov, const double* cov_const) = 0;
  // The same with the engine's states placed at column off of a caller state
  // of dimension ld (block decomposition of a larger state).
  virtual sm_status result_device_placed(void*, void*, int, int) { return fail(SM_ESTATE, "not supported"); }
  virtual sm_status set_trajectory_placed(const void*, const void*, const double*, int, int) {
    return fail(SM_ESTATE, "not supported");
  }

  // Per-track deltas (and their maximum, entry ntracks) of the last iteration,
  // read through a pinned host buffer.
  virtual sm_status track_deltas(double* out) {
    hipError_t e = hipSuccess;
    // an engine on an arena allocates nothing, pinned host memory included
    std::vector<unsigned long long> pageable(arena ? ntracks + 1 : 0);
    if (!h_delta && !arena)
      e = hipHostMalloc(reinterpret_cast<void**>(&h_delta), sizeof(unsigned long long) * (ntracks + 1),
                        hipHostMallocDefault);
    unsigned long long* host = arena ? pageable.data() : h_delta;
    if (e == hipSuccess)
      e = hipMemcpyAsync(host, delta_bits, sizeof(unsigned long long) * (ntracks + 1), hipMemcpyDeviceToHost,
                         stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "copy of the convergence statistic"));
    for (int i = 0; i <= ntracks; ++i) std::memcpy(&out[i], &host[i], sizeof(double));
    return SM_OK;
  }

  // Iterations until every track's delta has been below tol once, or max_iter
  // iterations.  first[i] = iteration (1-based, this call) at which track i
  // first fell below tol, 0 if it did not.
  // A track whose delta turns non-finite has failed: it is no longer waited
  // for (its first[] stays 0), the other tracks -- unaffected by it, since
  // track boundaries restart both scans -- run on, and the call then reports
  // SM_ENUMERIC.
  //
  // With freeze (engines where can_freeze()), a track that has converged or
  // failed is taken out of the later iterations: its trajectory stays the
  // iterate of that iteration, and tiles whose tracks are all out are
  // skipped.  Every track is put back in at the end of the call.
  sm_status iterate_until(double tol, int max_iter, int* run, int32_t* first, bool freeze = false) {
    std::vector<double> d(ntracks + 1);
    std::vector<unsigned char> failed(ntracks, 0), out(ntracks, 0);
    int left = ntracks, n_failed = 0;
    for (int i = 0; i < ntracks; ++i) first[i] = 0;
    *run = 0;
    freeze = freeze && can_freeze();
    sm_status st = freeze ? set_frozen(nullptr) : SM_OK;
    while (st == SM_OK && *run < max_iter && left > 0) {
      st = iterate(1);
      if (st == SM_OK) st = track_deltas(d.data());
      if (st != SM_OK) break;
      *run += 1;
      bool changed = false;
      for (int i = 0; i < ntracks; ++i) {
        if (failed[i] || out[i]) continue;
        if (!std::isfinite(d[i])) {
          // a track that had converged and then fails is reported as failed
          failed[i] = 1;
          ++n_failed;
          if (first[i] == 0) --left;
          first[i] = 0;
          out[i] = freeze;
          changed = changed || freeze;
        } else if (first[i] == 0 && d[i] < tol) {
          first[i] = *run;
          --left;
          out[i] = freeze;
          changed = changed || freeze;
        }
      }
      if (changed && left > 0) st = set_frozen(out.data());
    }
    if (freeze) {
      const sm_status st2 = set_frozen(nullptr);
      if (st == SM_OK) st = st2;
    }
    if (st != SM_OK) return st;
    if (n_failed > 0) return fail(SM_ENUMERIC, "non-finite iterate in " + std::to_string(n_failed) + " track(s)");
    return SM_OK;
  }

  // Per-track freeze mask for iterate_until (nullptr: no track frozen).
  virtual sm_status set_frozen(const unsigned char*) { return fail(SM_ESTATE, "freezing is not built for this engine"); }
  virtual bool can_freeze() const { return false; }

  // MAP objective (Section 3) of the current trajectory, per track, into a
  // host buffer; waits for the stream.
  virtual sm_status objective(double*) {
    return fail(SM_EINVAL, "the MAP objective is not built for this engine");
  }

  // One filtering pass linearised at the current trajectory, without damping:
  // filtered moments of every slot (host, nullable) and log p(y_{1:T}) of the
  // linearised model per track (nullable).  The trajectory, the iteration
  // count and the per-track deltas are left as they are.
  virtual sm_status filter(double*, double*, double*) {
    return fail(SM_EINVAL, "the filtering pass is not built for this engine");
  }

  // Levenberg-Marquardt hooks: per-track damping values replace the problem's
  // lm_lambda while the mode is on; save/restore keep the trajectory of the
  // tracks whose damped step is not taken.
  virtual sm_status lm_mode(bool) { return fail(SM_EINVAL, "adaptive damping is not built for this engine"); }
  virtual sm_status lm_set_lambda(const double*) { return fail(SM_ESTATE, "adaptive damping is off"); }
  virtual sm_status lm_save() { return fail(SM_ESTATE, "adaptive damping is off"); }
  virtual sm_status lm_restore(const unsigned char*) { return fail(SM_ESTATE, "adaptive damping is off"); }

  // Levenberg-Marquardt iterations with Marquardt's schedule, per track: a
  // damped pass with the track's lambda; the step is kept when the objective
  // does not rise by more than accept_rtol |J| (then lambda /= nu), otherwise
  // the trajectory is put back (lambda = min(lambda nu, kLmLambdaMax)).  A track
  // has converged at the first kept step whose largest change is below tol
  // while its lambda is at most lam0.  Runs until every track has converged or
  // max_iter iterations; first[i] as in iterate_until, cost[i] (nullable) the
  // final objective.
  sm_status iterate_lm(double lam0, double nu, double tol, int max_iter, double accept_rtol, int* run,
                       int32_t* first, double* cost) {
    sm_status st = lm_mode(true);
    if (st != SM_OK) return st;
    std::vector<double> lam(ntracks, lam0), J(ntracks), Jn(ntracks), d(ntracks + 1);
    std::vector<unsigned char> reject(ntracks, 0);
    for (int i = 0; i < ntracks; ++i) first[i] = 0;
    *run = 0;
    int left = ntracks, n_failed = 0;
    st = objective(J.data());
    // a track whose kept objective is not finite cannot recover (a pass is
    // kept only when its objective does not rise): it has failed and is not
    // waited for; a non-finite trial pass is simply rejected
    if (st == SM_OK)
      for (int i = 0; i < ntracks; ++i)
        if (!std::isfinite(J[i])) {
          ++n_failed;
          --left;
        }
    while (st == SM_OK && *run < max_iter && left > 0) {
      st = lm_set_lambda(lam.data());
      if (st == SM_OK) st = lm_save();
      if (st == SM_OK) st = iterate(1);
      if (st == SM_OK) st = objective(Jn.data());
      if (st == SM_OK) st = track_deltas(d.data());
      if (st != SM_OK) break;
      *run += 1;
      bool any = false;
      for (int i = 0; i < ntracks; ++i) {
        const bool taken = Jn[i] <= J[i] + accept_rtol * std::fabs(J[i]);
        reject[i] = taken ? 0 : 1;
        any = any || !taken;
        if (taken) {
          if (first[i] == 0 && d[i] < tol && lam[i] <= lam0) {
            first[i] = *run;
            --left;
          }
          J[i] = Jn[i];
          lam[i] /= nu;
        } else {
          lam[i] = std::min(lam[i] * nu, kLmLambdaMax);
        }
      }
      if (any) st = lm_restore(reject.data());
    }
    const sm_status off = lm_mode(false);
    if (st == SM_OK) st = off;
    if (cost)
      for (int i = 0; i < ntracks; ++i) cost[i] = J[i];
    if (st == SM_OK && n_failed > 0)
      return fail(SM_ENUMERIC, "non-finite objective in " + std::to_string(n_failed) + " track(s)");
    return st;
  }

  // Per-launch HIP events (only while profiling).  With prof_repeat > 1 each
  // launch runs that many times back to back between its event pair, which
  // spreads the latency of the event records and of the dispatch over the
  // repeats.  A kernel that computes its outputs from buffers it does not
  // write leaves after a repeat what it leaves after one launch (the
  // per-track change statistic is an atomic maximum); a kernel that
  // overwrites its own input passes repeatable = false and runs once.
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
    int64_t positions;
    int reps;
  };

  template <class F>
  void timed(const char* name, int64_t positions, F&& launch, bool repeatable = true) {
    if (!profiling) {
      launch();
      return;
    }
    const int reps = repeatable ? prof_repeat : 1;
    ProfRec r{name, nullptr, nullptr, positions, reps};
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, stream);
    for (int i = 0; i < reps; ++i) launch();
    (void)hipEventRecord(r.b, stream);
    prof.push_back(r);
  }

  virtual sm_status profile(int k, int repeat, sm_kernel_time* out, int cap_out, int* n_out) {
    prof.clear();
    prof_repeat = std::max(1, repeat);
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
      it->total_ms += ms / r.reps;
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

  // Device memory of the plan: one hipMalloc per buffer, or, once use_arena
  // has been called, 256-byte-aligned pieces of that caller-owned region
  // (never freed by the engine).
  void use_arena(void* base, size_t bytes) {
    arena = static_cast<char*>(base);
    arena_bytes = bytes;
    arena_used = 0;
  }

  hipError_t dalloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    if (cap > 0 && int64_t(device_bytes + bytes) > cap) return hipErrorOutOfMemory;
    if (arena) {
      const size_t off = (arena_used + 255) & ~size_t(255);
      if (off > arena_bytes || bytes > arena_bytes - off) return hipErrorOutOfMemory;
      *p = arena + off;
      arena_used = off + bytes;
      device_bytes += bytes;
      return hipSuccess;
    }
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
    if (h_delta) (void)hipHostFree(h_delta);
    h_delta = nullptr;
  }

  std::string err;
  int sched_lanes = 0, sched_slots = 0;
  int64_t sched_tiles = 0;
  int64_t S = 0;
  size_t stride = 0;
  int ntracks = 0;
  int n_iter = 0;
  int iters = 0;
  int64_t cap = 0;
  size_t device_bytes = 0;
  hipStream_t stream = nullptr;
  unsigned long long* delta_bits = nullptr;
  unsigned long long* h_delta = nullptr;   // pinned host copy of delta_bits
  std::vector<void*> allocs;
  bool freeze_converged = false;   // iterate_until takes converged tracks out (sm_problem)
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  bool profiling = false;
  int prof_repeat = 1;
  std::vector<ProfRec> prof;
};

// Factories, one per translation unit; nullptr for (nx, ny) not compiled.
EngineBase* make_engine_ct_f64(int nx, int ny);
EngineBase* make_engine_ct_f32(int nx, int ny);
EngineBase* make_engine_linear_f64(int nx, int ny);
EngineBase* make_engine_linear_f32(int nx, int ny);
EngineBase* make_engine_dense_ct_f64(int nx, int ny);
EngineBase* make_engine_dense_ct_f32(int nx, int ny);

}  // namespace pks
