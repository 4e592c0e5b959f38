// Host-side engine interface shared by the C ABI and the per-model
// translation units that instantiate the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
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

// Everything that depends on the model, dimensions and precision sits behind this interface.
class EngineBase {
 public:
  virtual ~EngineBase() { release(); }
  virtual sm_status setup(const sm_problem& pb, hipStream_t stream) = 0;
  virtual sm_status iterate(int k) = 0;
  virtual sm_status result_host(double* mean, double* cov) = 0;
  virtual sm_status result_device(void* mean, void* cov) = 0;
  virtual sm_status set_trajectory_device(const void* mean, const void* cov, const double* cov_const) = 0;

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
  std::vector<void*> allocs;
  bool profiling = false;
  std::vector<ProfRec> prof;
};

// Factories, one per translation unit; nullptr for (nx, ny) not compiled.
EngineBase* make_engine_ct_f64(int nx, int ny);
EngineBase* make_engine_ct_f32(int nx, int ny);
EngineBase* make_engine_linear_f64(int nx, int ny);
EngineBase* make_engine_linear_f32(int nx, int ny);

}  // namespace pks
