// Measurement kernels for the nx = 20 engine's wave routines (a separate
// library, libdense_probe.so; nothing in libsmoother.so calls it).
//
// Products.  The engine multiplies 20 x 20 FP64 matrices held in LDS, one
// wavefront per slot, with dn::mm: v_mfma_f64_16x16x4f64 on the product
// padded to 32 x 32, 2 x 2 output tiles of 16 x 16, 5 steps of 4 along the
// reduction, 20 MFMA per product (2.56 times the useful flops; MI355X's FP64
// matrix peak equals its FP64 vector peak).  The alternative is the VALU
// routine dn::mm_valu (each lane a 2 x 4 block of the result).  Both kernels
// below take the engine's LDS layout and accumulate C = reps * A B, one
// wavefront per block, so their durations compare the two forms directly.
//
// MFMA operand layout (lane l): A[l % 16][l / 16], B[l / 16][l % 16]; result
// element q of lane l is D[4 q + l / 16][l % 16], q = 0..3 (measured with
// one-hot operands: unlike the 16 x 16 x 16 BF16 form, consecutive result
// elements of a lane are rows 4 apart).
//
// Phases.  k_phases times the routines one filtering combine is made of
// (copy, Cholesky, products, triangular solve, symmetrisation) and the whole
// eq. 15 combine, its carry application and the eq. 19 combine, on seeded
// well-conditioned operands, with the shader clock (s_memtime) read by lane 0
// around each call: per block, the sum over `reps` calls of each.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dense.hpp"

namespace dprobe {

constexpr int N = 20;
constexpr int L = pks::dn::ld<N>();   // the engine's LDS row length

__device__ void stage(const double* A, const double* B, double* a, double* b) {
  const size_t off = size_t(blockIdx.x) * N * N;
  for (int e = threadIdx.x; e < N * N; e += 64) {
    a[(e / N) * L + e % N] = A[off + e];
    b[(e / N) * L + e % N] = B[off + e];
  }
  __syncthreads();
}

__global__ __launch_bounds__(64) void k_products_valu(const double* A, const double* B, double* C, int reps) {
  __shared__ double a[N * L], b[N * L], c[N * L];
  stage(A, B, a, b);
  for (int e = threadIdx.x; e < N * L; e += 64) c[e] = 0.0;
  __syncthreads();
  for (int r = 0; r < reps; ++r) pks::dn::mm_valu<N, N, N, N, false, false, double>(a, b, c, 1.0, c);
  const size_t off = size_t(blockIdx.x) * N * N;
  for (int e = threadIdx.x; e < N * N; e += 64) C[off + e] = c[(e / N) * L + e % N];
}

__global__ __launch_bounds__(64) void k_products_mfma(const double* A, const double* B, double* C, int reps) {
  __shared__ double a[N * L], b[N * L], c[N * L];
  stage(A, B, a, b);
  for (int e = threadIdx.x; e < N * L; e += 64) c[e] = 0.0;
  __syncthreads();
  for (int r = 0; r < reps; ++r) pks::dn::mm<N, N, N, N, false, false, double>(a, b, c, 1.0, c);
  const size_t off = size_t(blockIdx.x) * N * N;
  for (int e = threadIdx.x; e < N * N; e += 64) C[off + e] = c[(e / N) * L + e % N];
}

constexpr int kPhases = 11;

// Symmetric positive definite test matrix, diagonally dominant: diag on the
// diagonal, off / (1 + |i - j|) elsewhere; the padding column is zero.
__device__ void spd(double* M, double diag, double off) {
  for (int e = threadIdx.x; e < N * L; e += 64) {
    const int i = e / L, j = e % L;
    M[e] = j >= N ? 0.0 : (i == j ? diag : off / (1.0 + (i > j ? i - j : j - i)));
  }
}

__global__ __launch_bounds__(64) void k_phases(unsigned long long* out, int reps) {
  using pks::dn::Work;
  __shared__ Work<N, double, 9> w;
  __shared__ double keep[N * L];
  double *lA = w.m[0], *lC = w.m[1], *lJ = w.m[2], *rA = w.m[3], *rC = w.m[4], *rJ = w.m[5];
  double *T1 = w.m[6], *T2 = w.m[7], *T3 = w.m[8];
  if (threadIdx.x == 0) w.ok = 1;
  unsigned long long acc[kPhases];
  for (int p = 0; p < kPhases; ++p) acc[p] = 0ull;
  for (int r = 0; r < reps; ++r) {
    spd(lA, 0.5, 0.05);
    spd(lC, 2.0, 0.3);
    spd(lJ, 1.5, 0.2);
    spd(rA, 0.6, 0.04);
    spd(rC, 1.8, 0.25);
    spd(rJ, 1.2, 0.1);
    spd(keep, 2.0, 0.3);
    for (int i = threadIdx.x; i < N; i += 64) {
      w.v[0][i] = 0.1 * i;
      w.v[1][i] = 0.2;
      w.v[2][i] = -0.1;
      w.v[3][i] = 0.3;
    }
    __syncthreads();
    unsigned long long t0, t1;
#define PHASE(p, call)                   \
    t0 = __builtin_amdgcn_s_memtime();   \
    call;                                \
    t1 = __builtin_amdgcn_s_memtime();   \
    acc[p] += t1 - t0;
    PHASE(0, (pks::dn::copy<N, N, N, false>(keep, T1)))
    PHASE(1, (pks::dn::chol<N, N>(T1, &w.ok)))
    PHASE(2, (pks::dn::mm<N, N, N, N, false, false>(rJ, T1, (const double*)nullptr, 1.0, T2)))
    PHASE(3, (pks::dn::mm<N, N, N, N, true, false>(T1, T2, (const double*)nullptr, 1.0, T3)))
    PHASE(4, (pks::dn::copy<N, N, N, true>(T1, T2)))
    PHASE(5, (pks::dn::fwd<N, N, N>(T1, T2)))
    PHASE(6, (pks::dn::mv<N, N, N, false>(rJ, w.v[0], w.v[1], -1.0, w.v[4])))
    PHASE(7, (pks::dn::symmetrize<N, N>(lJ)))
    pks::dn::copy<N, N, N, false>(rJ, T3);   // the combine destroys its J operand
    PHASE(8, (pks::dn::combine_f<N, double>(lA, w.v[0], lC, w.v[1], lJ, rA, w.v[2], rC, w.v[3], T3, T1, T2, w.v[4],
                                             w.v[5], &w.ok)))
    pks::dn::copy<N, N, N, false>(rJ, T3);   // apply_f destroys its J operand
    spd(lC, 2.0, 0.3);
    __syncthreads();
    PHASE(9, (pks::dn::apply_f<N, double>(w.v[0], lC, rA, w.v[2], rC, w.v[3], T3, T1, w.v[4], w.v[5], &w.ok)))
    spd(lA, 0.5, 0.05);
    __syncthreads();
    PHASE(10, (pks::dn::combine_s<N, double>(lA, w.v[0], lC, rA, w.v[2], rC, T1, T2, w.v[4])))
#undef PHASE
  }
  if (threadIdx.x == 0)
    for (int p = 0; p < kPhases; ++p) out[size_t(blockIdx.x) * kPhases + p] = acc[p];
}

}  // namespace dprobe

extern "C" {

// C[b] = reps * A[b] B[b] for b < blocks (device FP64, [blocks][20][20] each,
// row-major), variant 0 = VALU (dn::mm_valu), 1 = the engine's FP64 MFMA
// routine (dn::mm), on the given HIP stream (null = default).  Returns the
// launch's hipError_t.
int dprobe_products(int variant, int blocks, int reps, const double* A, const double* B, double* C,
                    void* stream) {
  if (blocks < 1 || reps < 1 || !A || !B || !C || (variant != 0 && variant != 1)) return int(hipErrorInvalidValue);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (variant == 0)
    hipLaunchKernelGGL(dprobe::k_products_valu, dim3(unsigned(blocks)), dim3(64), 0, s, A, B, C, reps);
  else
    hipLaunchKernelGGL(dprobe::k_products_mfma, dim3(unsigned(blocks)), dim3(64), 0, s, A, B, C, reps);
  return int(hipGetLastError());
}

// Number of routines k_phases times.
int dprobe_phase_count(void) { return dprobe::kPhases; }

// Shader-clock cycles of the nx = 20 wave routines: out (device, [blocks]
// [dprobe_phase_count()] unsigned 64-bit) receives per block the sum over
// `reps` calls of each routine, in the order copy, Cholesky, product,
// product with A transposed, transposed copy, forward substitution with 20
// right-hand sides, matrix-vector product, symmetrisation, eq. 15 combine,
// carry application, eq. 19 combine.  Returns the launch's hipError_t.
int dprobe_phases(int blocks, int reps, unsigned long long* out, void* stream) {
  if (blocks < 1 || reps < 1 || !out) return int(hipErrorInvalidValue);
  hipLaunchKernelGGL(dprobe::k_phases, dim3(unsigned(blocks)), dim3(64), 0, static_cast<hipStream_t>(stream), out,
                     reps);
  return int(hipGetLastError());
}

}  // extern "C"
