// Host stand-in for <hip/hip_runtime.h>: just enough to compile the
// library's per-lane device algebra (linalg.hpp, operators.hpp, sqrt.hpp,
// elements.hpp, models.hpp) as plain C++ for a host build under
// AddressSanitizer and UndefinedBehaviorSanitizer.  Cross-lane operations are
// not modelled: functions that use them are never instantiated here.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)

using std::atan2;
using std::fabs;
using std::floor;
using std::fma;
using std::sqrt;

inline void sincos(double x, double* s, double* c) {
  *s = std::sin(x);
  *c = std::cos(x);
}
inline void sincosf(float x, float* s, float* c) {
  *s = std::sin(x);
  *c = std::cos(x);
}

// The hardware estimates are stood in for by the exact values; the library
// refines them by Newton steps, which leave an exact value in place.
inline double __builtin_amdgcn_rsq(double x) { return 1.0 / std::sqrt(x); }
inline float __builtin_amdgcn_rsqf(float x) { return 1.0f / std::sqrt(x); }
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
inline float __builtin_amdgcn_rcpf(float x) { return 1.0f / x; }

template <typename T>
T __shfl(T v, int) {
  return v;
}
