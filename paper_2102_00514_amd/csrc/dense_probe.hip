// Measurement kernels for the nx = 20 engine's level-0 matrix products (a
// separate library, libdense_probe.so; nothing in libsmoother.so calls it).
//
// The engine multiplies 20 x 20 FP64 matrices held in LDS, one wavefront per
// slot, with the VALU routine dn::mm (each lane a 2 x 4 block of the result).
// The alternative on the matrix cores is v_mfma_f64_16x16x4f64: the product
// padded to 32 x 32, 2 x 2 output tiles of 16 x 16, 5 steps of 4 along the
// reduction, 20 MFMA per product (2.56 times the useful flops; MI355X's FP64
// matrix peak equals its FP64 vector peak).  Both kernels below take the same
// LDS layout as the engine and accumulate C = reps * A B, one wavefront per
// block, so their durations compare the two forms directly.
//
// MFMA operand layout (lane l): A[l % 16][l / 16], B[l / 16][l % 16]; result
// element q of lane l is D[4 q + l / 16][l % 16], q = 0..3 (measured with
// one-hot operands: unlike the 16 x 16 x 16 BF16 form, consecutive result
// elements of a lane are rows 4 apart).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dense.hpp"

namespace dprobe {

constexpr int N = 20;
constexpr int L = pks::dn::ld<N>();   // the engine's LDS row length
typedef double f64x4 __attribute__((ext_vector_type(4)));

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
  for (int r = 0; r < reps; ++r) pks::dn::mm<N, N, N, N, false, false, double>(a, b, c, 1.0, c);
  const size_t off = size_t(blockIdx.x) * N * N;
  for (int e = threadIdx.x; e < N * N; e += 64) C[off + e] = c[(e / N) * L + e % N];
}

__global__ __launch_bounds__(64) void k_products_mfma(const double* A, const double* B, double* C, int reps) {
  __shared__ double a[N * L], b[N * L];
  stage(A, B, a, b);
  const int r = threadIdx.x & 15, kq = threadIdx.x >> 4;
  f64x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int rep = 0; rep < reps; ++rep) {
#pragma unroll
    for (int ks = 0; ks < 5; ++ks) {
      const int k = 4 * ks + kq;   // < 20
      double av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = 16 * t + r;
        av[t] = i < N ? a[i * L + k] : 0.0;
        bv[t] = i < N ? b[k * L + i] : 0.0;
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
  }
  const size_t off = size_t(blockIdx.x) * N * N;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * ti + 4 * q + kq, j = 16 * tj + r;
        if (i < N && j < N) C[off + size_t(i) * N + j] = acc[ti][tj][q];
      }
}

}  // namespace dprobe

extern "C" {

// C[b] = reps * A[b] B[b] for b < blocks (device FP64, [blocks][20][20] each,
// row-major), variant 0 = VALU (the engine's routine), 1 = FP64 MFMA, on the
// given HIP stream (null = default).  Returns the launch's hipError_t.
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

}  // extern "C"
