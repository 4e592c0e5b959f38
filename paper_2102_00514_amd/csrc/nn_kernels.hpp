// Kernels of the warm-start network: a patch-embedding 1-D convolution,
// dilated residual convolutions and a per-patch linear head, FP32, with the
// backward pass and Adam.  Activations are channel-major, [channels][n * L]
// (window-major positions inside a channel row), so every convolution is a
// GEMM whose right operand is gathered on the fly from the source rows.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wsn {

constexpr int kTile = 64;     // output rows and columns per block
constexpr int kTk = 16;       // reduction depth staged per LDS step
constexpr int kThreads = 256; // 16 x 16 threads, 4 x 4 outputs each
constexpr int kPad = 4;       // LDS row padding: column writes of 16 rows hit distinct banks

// B(r, p) of a convolution: r = c * K + k (source row c, tap k), p = w * Lout + j
// (window w, output position j); the source position is j * stride + k * dil - pad,
// zero outside [0, Lin).
struct Gather {
  const float* src;  // [rows][ld]
  int ld;            // n * Lin
  int K, Lout, Lin, stride, dil, pad;
};

__device__ __forceinline__ float gather_at(const Gather& g, int r, int p) {
  const int c = r / g.K, k = r - c * g.K;
  const int w = p / g.Lout, j = p - w * g.Lout;
  const int s = j * g.stride + k * g.dil - g.pad;
  return (s >= 0 && s < g.Lin) ? g.src[size_t(c) * g.ld + size_t(w) * g.Lin + s] : 0.f;
}

enum Epilogue { kEpiRelu = 0, kEpiResidual = 1, kEpiLinear = 2, kEpiBackward = 3 };

struct ConvArgs {
  int M, Kr, N;          // output rows, reduction length, output positions (N % 4 == 0)
  const float* W;        // weights [Cout][Cin][K]
  int transposed;        // 0: A(m, r) = W[m * Kr + r]; 1: A(m, r = co * K + k) = W[(co * M + m) * K + k]
  const float* bias;     // [M] (forward epilogues)
  Gather g;
  float* out;            // relu: h; residual: relu part a; linear: output; backward: dh (nullable)
  float* out2;           // residual: h_prev + a; backward: dh masked by (mask > 0)
  const float* in2;      // residual: h_prev; backward: dh of the layer above (nullable)
  const float* mask;     // backward: relu output of the source layer
};

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

// One reduction stage of a 64 x 64 output tile: As[rr][mm] = A(m0 + mm, r0 + rr),
// Bs[rb][pp] = B(r0 + rb, p0 + pp), zero outside the matrices.
__device__ __forceinline__ void stage_tile(const ConvArgs& a, int t, int m0, int p0, int r0,
                                           float (&As)[kTk][kTile + kPad], float (&Bs)[kTk][kTile]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = t + kThreads * i;
    // weights: consecutive lanes take consecutive addresses of W in both forms
    if (a.transposed) {
      const int mm = e & 63, rr = e >> 6, m = m0 + mm, r = r0 + rr;
      float v = 0.f;
      if (m < a.M && r < a.Kr) {
        const int co = r / a.g.K, k = r - co * a.g.K;
        v = a.W[(size_t(co) * a.M + m) * a.g.K + k];
      }
      As[rr][mm] = v;
    } else {
      const int rr = e & 15, mm = e >> 4, m = m0 + mm, r = r0 + rr;
      As[rr][mm] = (m < a.M && r < a.Kr) ? a.W[size_t(m) * a.Kr + r] : 0.f;
    }
    const int pp = e & 63, rb = e >> 6, p = p0 + pp, r = r0 + rb;
    Bs[rb][pp] = (p < a.N && r < a.Kr) ? gather_at(a.g, r, p) : 0.f;
  }
}

// out[m][p] = epilogue(sum_r A(m, r) B(r, p)); grid (ceil(N / 64), ceil(M / 64)).
template <int EPI>
__global__ __launch_bounds__(kThreads) void k_conv(ConvArgs a) {
  __shared__ __align__(16) float As[kTk][kTile + kPad];
  __shared__ __align__(16) float Bs[kTk][kTile];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int m0 = blockIdx.y * kTile, p0 = blockIdx.x * kTile;
  float acc[4][4] = {};
  for (int r0 = 0; r0 < a.Kr; r0 += kTk) {
    stage_tile(a, t, m0, p0, r0, As, Bs);
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kTk; ++rr) {
      const float4 av = ld4(&As[rr][4 * ty]);
      const float4 bv = ld4(&Bs[rr][4 * tx]);
      const float ar[4] = {av.x, av.y, av.z, av.w};
      const float br[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(ar[i], br[j], acc[i][j]);
    }
    __syncthreads();
  }
  const int p = p0 + 4 * tx;
  if (p >= a.N) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + 4 * ty + i;
    if (m >= a.M) break;
    const size_t o = size_t(m) * a.N + p;
    float4 v = make_float4(acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
    if (EPI == kEpiBackward) {
      if (a.in2) {
        const float4 u = ld4(a.in2 + o);
        v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
      }
      if (a.out) st4(a.out + o, v);
      const float4 mk = ld4(a.mask + o);
      st4(a.out2 + o, make_float4(mk.x > 0.f ? v.x : 0.f, mk.y > 0.f ? v.y : 0.f,
                                  mk.z > 0.f ? v.z : 0.f, mk.w > 0.f ? v.w : 0.f));
    } else {
      const float b = a.bias[m];
      v.x += b; v.y += b; v.z += b; v.w += b;
      if (EPI == kEpiLinear) {
        st4(a.out + o, v);
      } else {
        v = make_float4(fmaxf(v.x, 0.f), fmaxf(v.y, 0.f), fmaxf(v.z, 0.f), fmaxf(v.w, 0.f));
        st4(a.out + o, v);
        if (EPI == kEpiResidual) {
          const float4 u = ld4(a.in2 + o);
          st4(a.out2 + o, make_float4(u.x + v.x, u.y + v.y, u.z + v.z, u.w + v.w));
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Inference form of the forward convolutions on the matrix cores: the same
// tiles and staging as k_conv, the products as 16 x 16 x 16 BF16 MFMA with
// FP32 accumulation (operands rounded to BF16, to nearest even).  Each of the
// four waves owns a 32 x 32 quarter of the 64 x 64 tile, two by two MFMA
// blocks.  Operand layout of the MFMA (lane l, element j): A[l % 16][4 (l / 16)
// + j], B[4 (l / 16) + j][l % 16]; result D[4 (l / 16) + j][l % 16].
// Forward epilogues only (bias + ReLU, residual, linear).
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return short(u >> 16);
}

template <int EPI>
__global__ __launch_bounds__(kThreads) void k_conv_mfma(ConvArgs a) {
  static_assert(EPI != kEpiBackward, "forward epilogues only");
  __shared__ __align__(16) float As[kTk][kTile + kPad];
  __shared__ __align__(16) float Bs[kTk][kTile];
  const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
  const int m0 = blockIdx.y * kTile, p0 = blockIdx.x * kTile;
  const int mw = (wv >> 1) * 32, nw = (wv & 1) * 32;   // this wave's quarter of the tile
  const int kq = 4 * (ln >> 4), lr = ln & 15;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int r0 = 0; r0 < a.Kr; r0 += kTk) {
    stage_tile(a, t, m0, p0, r0, As, Bs);
    __syncthreads();
    bf16x4 af[2], bf[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        af[i][j] = to_bf16(As[kq + j][mw + 16 * i + lr]);
        bf[i][j] = to_bf16(Bs[kq + j][nw + 16 * i + lr]);
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bf[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + mw + 16 * i + kq + q, p = p0 + nw + 16 * j + lr;
        if (m >= a.M || p >= a.N) continue;
        const size_t o = size_t(m) * a.N + p;
        float v = acc[i][j][q] + a.bias[m];
        if (EPI == kEpiLinear) {
          a.out[o] = v;
        } else {
          v = fmaxf(v, 0.f);
          a.out[o] = v;
          if (EPI == kEpiResidual) a.out2[o] = a.in2[o] + v;
        }
      }
}

// ---------------------------------------------------------------------------
// Inference form of a dilated residual layer, h' = h + relu(b + sum_k W_k h(.
// + (k - 1) d)), for C channels in and out (C = 128 or 256).  A block takes
// 128 positions -- whole windows, so every tap that stays inside its window
// stays inside the tile -- and all C output channels.  Its input tile is read
// from HBM once, rounded to BF16 and staged position-major in LDS, where one
// 8-byte read gives an MFMA B fragment (4 consecutive channels at one
// position); the packed weights give A fragments the same way.  The residual
// is added from the unrounded FP32 input, and only h' is written (the ReLU
// part alone is kept by the training form, for the backward pass).
// Wave w computes rows 32 w .. 32 w + 31 of each 128-row chunk, all 128
// positions: 2 x 8 blocks of 16 x 16 x 16 BF16 MFMA, FP32 accumulation.
// grid ceil(N / 128); requires 128 % Lpos == 0 and N % Lpos == 0.
// ---------------------------------------------------------------------------
struct ResidualArgs {
  int N, Lpos, dil;     // positions, positions per window, dilation
  const short* Wt;      // [C][3][C] BF16 bits: Wt[(m * 3 + k) * C + c] = bf16(W[m][c][k])
  const float* bias;    // [C]
  const float* h;       // [C][N] layer input
  float* out;           // [C][N] layer output h'
};

constexpr int kResP = 128;   // positions per block of k_residual_mfma

// Wt[(m * 3 + k) * C + c] = bf16(W[(m * C + c) * 3 + k]); grid ceil(3 C^2 / 256).
__global__ __launch_bounds__(256) void k_pack_residual(const float* W, int C, short* Wt) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= int64_t(3) * C * C) return;
  const int c = int(e % C), k = int((e / C) % 3);
  const int64_t m = e / (int64_t(3) * C);
  Wt[e] = to_bf16(W[(m * C + c) * 3 + k]);
}

template <int C>
__global__ __launch_bounds__(256) void k_residual_mfma(ResidualArgs a) {
  static_assert(C % 128 == 0, "128-row chunks");
  constexpr int CP = C + 8;   // LDS row pitch (BF16): rows 16 B apart in bank order
  __shared__ __align__(16) short Hs[kResP][CP];
  const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
  const int64_t p0 = int64_t(blockIdx.x) * kResP;
  // stage the tile: each thread moves 4 channels x 4 positions per pass
  // (float4 reads along positions, one 8-byte LDS write per position)
  for (int b = t; b < (C / 4) * (kResP / 4); b += 256) {
    const int cb = b / (kResP / 4), pb = b - cb * (kResP / 4);
    const int c = 4 * cb, p = 4 * pb;
    const int64_t pp = p0 + p;
    float v[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (pp + 3 < a.N) {
        const float4 x = ld4(a.h + int64_t(c + i) * a.N + pp);
        v[i][0] = x.x; v[i][1] = x.y; v[i][2] = x.z; v[i][3] = x.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[i][j] = pp + j < a.N ? a.h[int64_t(c + i) * a.N + pp + j] : 0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf16x4 w;
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] = to_bf16(v[i][j]);
      *reinterpret_cast<bf16x4*>(&Hs[p + j][c]) = w;
    }
  }
  __syncthreads();
  const int kq = 4 * (ln >> 4), lr = ln & 15;
  for (int m0 = 0; m0 < C; m0 += 128) {
    const int mrow = m0 + 32 * wv + lr;   // A-fragment row of block i: mrow + 16 i
    f32x4 acc[2][8];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 3; ++k) {
      const int off = (k - 1) * a.dil;
      // per position block j: the tap's LDS row and whether it stays in the window
      int row[8];
      bool live[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int pl = 16 * j + lr, q = pl % a.Lpos + off;
        live[j] = q >= 0 && q < a.Lpos;
        row[j] = live[j] ? pl + off : pl;
      }
#pragma unroll 2
      for (int c0 = 0; c0 < C; c0 += 16) {
        bf16x4 af[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
          af[i] = *reinterpret_cast<const bf16x4*>(a.Wt + (int64_t(mrow + 16 * i) * 3 + k) * C + c0 + kq);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          bf16x4 bv = *reinterpret_cast<const bf16x4*>(&Hs[row[j]][c0 + kq]);
          if (!live[j]) bv = bf16x4{0, 0, 0, 0};
#pragma unroll
          for (int i = 0; i < 2; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bv, acc[i][j], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 32 * wv + 16 * i + kq + q;
        const float bm = a.bias[m];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t p = p0 + 16 * j + lr;
          if (p >= a.N) continue;
          const int64_t o = int64_t(m) * a.N + p;
          a.out[o] = a.h[o] + fmaxf(acc[i][j][q] + bm, 0.f);
        }
      }
  }
}

// Weight gradient partials: part[z][m][r] = sum over the z-th chunk of
// positions of D[m][p] B(r, p), with r = Kr the bias column (B = 1).
// grid (ceil((Kr + 1) / 64), ceil(M / 64), chunks).
struct WgradArgs {
  int M, Kr, N, chunk;
  const float* D;   // [M][N]
  Gather g;
  float* part;      // [chunks][M][Kr + 1]
};

__global__ __launch_bounds__(kThreads) void k_wgrad(WgradArgs a) {
  __shared__ __align__(16) float Ds[kTk][kTile + kPad];
  __shared__ __align__(16) float Bs[kTk][kTile + kPad];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int r0 = blockIdx.x * kTile, m0 = blockIdx.y * kTile;
  const int pbeg = blockIdx.z * a.chunk;
  const int pend = min(pbeg + a.chunk, a.N);
  const int R1 = a.Kr + 1;
  float acc[4][4] = {};
  for (int pc = pbeg; pc < pend; pc += kTk) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = t + kThreads * i, pp = e & 15, q = e >> 4;   // q: row (m or r) within the tile
      const int p = pc + pp;
      const bool live = p < pend;
      const int m = m0 + q;
      Ds[pp][q] = (live && m < a.M) ? a.D[size_t(m) * a.N + p] : 0.f;
      const int r = r0 + q;
      float bv = 0.f;
      if (live && r < R1) bv = r == a.Kr ? 1.f : gather_at(a.g, r, p);
      Bs[pp][q] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int pp = 0; pp < kTk; ++pp) {
      const float4 dv = ld4(&Ds[pp][4 * ty]);
      const float4 bv = ld4(&Bs[pp][4 * tx]);
      const float dr[4] = {dv.x, dv.y, dv.z, dv.w};
      const float br[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(dr[i], br[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + 4 * ty + i;
    if (m >= a.M) break;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + 4 * tx + j;
      if (r < R1) a.part[(size_t(blockIdx.z) * a.M + m) * R1 + r] = acc[i][j];
    }
  }
}

// Sums the chunk partials (in chunk order) into the flat gradient:
// W part at w_off + m * Kr + r, bias at b_off + m.
__global__ void k_wgrad_reduce(const float* part, int chunks, int M, int Kr, float* grad, int64_t w_off,
                               int64_t b_off) {
  const int R1 = Kr + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * R1) return;
  const int m = e / R1, r = e - m * R1;
  float s = 0.f;
  for (int z = 0; z < chunks; ++z) s += part[(size_t(z) * M + m) * R1 + r];
  if (r < Kr) grad[w_off + size_t(m) * Kr + r] = s;
  else grad[b_off + m] = s;
}

// Mean-squared error: dout = scale * (out - target), scale = 2 / count; block
// partial sums of the squared error (fixed order) into part[blockIdx.x].
__global__ __launch_bounds__(256) void k_mse(const float* out, const float* target, float* dout, int64_t count,
                                             float scale, float* part) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < count; e += int64_t(gridDim.x) * 256) {
    const float d = out[e] - target[e];
    dout[e] = scale * d;
    s = fmaf(d, d, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum(const float* part, int n, float scale, float* out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int e = threadIdx.x; e < n; e += 256) s += part[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

// Adam (Kingma & Ba, 2015) with bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_adam(float* theta, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = beta1 * m[e] + (1.f - beta1) * gi;
  const float vi = beta2 * v[e] + (1.f - beta2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  theta[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Windows of the planned tracks (device tables).
struct WindowTable {
  const int* track;        // [n_windows] track of each window
  const int* start;        // [n_windows] first step (1-based) of each window
  const int64_t* meas_off; // [n_tracks + 1] measurement offsets
  const int* first;        // [n_tracks + 1] first window of each track
};

// Network inputs of windows w0 .. w0 + n - 1: (sin, cos) of every bearing.
// channel_major: x[c][b * W + t] (a batch), else x[b][c][t] (a data set).
__global__ void k_features(WindowTable tab, const double* y, int ny, int W, int64_t w0, int n, int channel_major,
                           float* x) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n) * W) return;
  const int b = int(e / W), t = int(e - int64_t(b) * W);
  const int64_t w = w0 + b;
  const int tr = tab.track[w];
  const int64_t T = tab.meas_off[tr + 1] - tab.meas_off[tr];
  const int64_t k = min(int64_t(tab.start[w]) + t, T);
  const double* yk = y + (tab.meas_off[tr] + k - 1) * ny;
  const int cin = 2 * ny;
  for (int s = 0; s < ny; ++s) {
    double sv, cv;
    sincos(yk[s], &sv, &cv);
    const size_t i0 = channel_major ? size_t(2 * s) * n * W + size_t(b) * W + t : (size_t(b) * cin + 2 * s) * W + t;
    const size_t i1 = channel_major ? i0 + size_t(n) * W : i0 + W;
    x[i0] = float(sv);
    x[i1] = float(cv);
  }
}

// Labels of every window from smoothed means [S][nx]: lab[w][t][i].
__global__ void k_labels(WindowTable tab, const double* mean, int nx, int W, int64_t n_windows, float* lab) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n_windows * W) return;
  const int64_t w = e / W;
  const int t = int(e - w * W);
  const int tr = tab.track[w];
  const int64_t T = tab.meas_off[tr + 1] - tab.meas_off[tr];
  const int64_t k = min(int64_t(tab.start[w]) + t, T);
  const int64_t slot = tab.meas_off[tr] + tr + k;
  for (int i = 0; i < nx; ++i) lab[e * nx + i] = float(mean[slot * nx + i]);
}

// Batch assembly from a data set of n_data windows: xb[c][b * W + t] =
// x[idx[b]][c][t]; when lab is given, tb[u * nx + i][b * L + j] =
// (lab[idx[b]][P j + u][i] - mu_i) / sigma_i.  An index outside [0, n_data)
// reads nothing: its window is zero and *bad is set.
__global__ void k_gather_batch(const float* x, const float* lab, int64_t n_data, const int* idx, int n, int cin,
                               int W, int P, int nx, const float* mu, const float* sigma, float* xb, float* tb,
                               int* bad) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n) * W) return;
  const int b = int(e / W), t = int(e - int64_t(b) * W);
  const int64_t src = idx[b];
  const bool ok = src >= 0 && src < n_data;
  if (!ok && t == 0) atomicOr(bad, 1);
  for (int c = 0; c < cin; ++c) xb[size_t(c) * n * W + e] = ok ? x[(src * cin + c) * W + t] : 0.f;
  if (lab) {
    const int L = W / P, j = t / P, u = t - j * P;
    for (int i = 0; i < nx; ++i)
      tb[size_t(u * nx + i) * n * L + size_t(b) * L + j] =
          ok ? (lab[(src * W + t) * nx + i] - mu[i]) / sigma[i] : 0.f;
  }
}

// Network outputs [P nx][n L] -> states out[b][t][i] = mu_i + sigma_i * o.
__global__ void k_states(const float* o, int n, int W, int P, int nx, const float* mu, const float* sigma,
                         float* out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n) * W) return;
  const int b = int(e / W), t = int(e - int64_t(b) * W);
  const int L = W / P, j = t / P, u = t - j * P;
  for (int i = 0; i < nx; ++i)
    out[e * nx + i] = mu[i] + sigma[i] * o[size_t(u * nx + i) * n * L + size_t(b) * L + j];
}

// Network outputs of windows w0 .. w0 + n - 1 -> initial trajectory mean[S][nx]
// (FP64): step k of a track comes from window min((k - 1) / W, n_w - 1) of that
// track, slot 0 from step 1.
__global__ void k_scatter(WindowTable tab, const float* o, int64_t w0, int n, int W, int P, int nx,
                          const float* mu, const float* sigma, double* mean) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n) * W) return;
  const int b = int(e / W), t = int(e - int64_t(b) * W);
  const int64_t w = w0 + b;
  const int tr = tab.track[w];
  const int64_t T = tab.meas_off[tr + 1] - tab.meas_off[tr];
  const int64_t k = int64_t(tab.start[w]) + t;
  if (k > T) return;
  const int nw = tab.first[tr + 1] - tab.first[tr];
  const int64_t owner = tab.first[tr] + min((k - 1) / W, int64_t(nw - 1));
  if (owner != w) return;
  const int L = W / P, j = t / P, u = t - j * P;
  const int64_t slot = tab.meas_off[tr] + tr + k;
  for (int i = 0; i < nx; ++i) {
    const double v = double(mu[i] + sigma[i] * o[size_t(u * nx + i) * n * L + size_t(b) * L + j]);
    mean[slot * nx + i] = v;
    if (k == 1) mean[(slot - 1) * nx + i] = v;
  }
}

}  // namespace wsn
