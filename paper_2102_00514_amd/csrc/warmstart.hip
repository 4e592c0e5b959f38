// C ABI of the warm-start network (warmstart.h): parameters, Adam state,
// workspace and the launch sequence of the forward and backward passes.
#include "warmstart.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "nn_kernels.hpp"

namespace {

thread_local std::string g_create_error;

struct LayerSpec {
  int cout, cin, K, stride, dil, pad;
  int64_t w_off, b_off;
  int64_t weights() const { return int64_t(cout) * cin * K; }
};

const char* check_config(const ws_config& c) {
  if (c.window < 4 || c.window > 4096) return "window must be in [4, 4096]";
  if (c.patch < 1 || c.window % c.patch != 0) return "patch must divide window";
  if ((c.window / c.patch) % 4 != 0) return "window / patch must be a multiple of 4";
  if (c.width < 1 || c.width > 4096) return "width must be in [1, 4096]";
  if (c.hidden < 0 || c.hidden > 12) return "hidden must be in [0, 12]";
  if (c.nx < 1 || c.nx > 64) return "nx must be in [1, 64]";
  if (c.ny < 1 || c.ny > 32) return "ny must be in [1, 32]";
  if (c.max_batch < 1 || int64_t(c.max_batch) * c.window > (int64_t(1) << 30))
    return "max_batch must be >= 1 with max_batch * window <= 2^30";
  return nullptr;
}

std::vector<LayerSpec> layer_specs(const ws_config& c) {
  std::vector<LayerSpec> L;
  L.push_back({c.width, 2 * c.ny, c.patch, c.patch, 1, 0, 0, 0});
  for (int l = 1; l <= c.hidden; ++l) {
    const int d = 1 << (l - 1);
    L.push_back({c.width, c.width, 3, 1, d, d, 0, 0});
  }
  L.push_back({c.patch * c.nx, c.width, 1, 1, 0, 0, 0, 0});
  int64_t off = 0;
  for (auto& s : L) {
    s.w_off = off;
    s.b_off = off + s.weights();
    off = s.b_off + s.cout;
  }
  return L;
}

int64_t total_params(const std::vector<LayerSpec>& L) { return L.back().b_off + L.back().cout; }

std::string hip_msg(hipError_t e, const char* what) { return std::string(what) + ": " + hipGetErrorString(e); }

constexpr int kWgradTarget = 512;  // blocks aimed at per weight-gradient launch

}  // namespace

struct ws_net {
  ws_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<LayerSpec> layers;
  int64_t n_params = 0;
  int64_t step = 0;
  int Lpos = 0;   // positions per window after the embedding
  std::vector<void*> allocs;
  float *theta = nullptr, *grad = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  float *mu = nullptr, *sigma = nullptr;
  float *xb = nullptr, *tb = nullptr, *out = nullptr, *dout = nullptr;
  std::vector<float*> H, A;   // H[0..hidden], A[1..hidden] (A[0] unused: h0 is its own relu output)
  float *dh[2] = {nullptr, nullptr}, *dz[2] = {nullptr, nullptr};
  float *part = nullptr, *loss_part = nullptr, *loss = nullptr;
  int* bad_index = nullptr;   // set by the batch gather when an index is out of range
  short* wt16 = nullptr;      // residual weights packed for k_residual_mfma ([hidden][3 C^2] BF16)
  bool res_fast = false;      // the inference form runs k_residual_mfma (C = 128 or 256, 128 % Lpos == 0)
  int64_t part_floats = 0;
  int* win_track = nullptr;
  int* win_start = nullptr;
  int* first = nullptr;
  int64_t* meas_off = nullptr;
  int64_t n_windows = 0;
  int n_tracks = 0;
  std::vector<void*> plan_allocs;

  ws_status fail(ws_status s, std::string msg) {
    err = std::move(msg);
    return s;
  }

  hipError_t alloc(void** p, size_t bytes, std::vector<void*>& list) {
    const hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e == hipSuccess) list.push_back(*p);
    return e;
  }

  ~ws_net() {
    for (void* p : plan_allocs) (void)hipFree(p);
    for (void* p : allocs) (void)hipFree(p);
  }

  wsn::WindowTable table() const { return {win_track, win_start, meas_off, first}; }

  // Chunks of the weight-gradient reduction for M x (Kr + 1) tiles over N
  // positions.  The result never exceeds wgrad_chunk_bound(M, Kr, N), which
  // grows with N, so a workspace sized by the bound at max_batch serves every batch.
  static int wgrad_chunk_bound(int M, int Kr, int N) {
    const int tiles = ((Kr + 1 + wsn::kTile - 1) / wsn::kTile) * ((M + wsn::kTile - 1) / wsn::kTile);
    return std::max(1, std::min((kWgradTarget + tiles - 1) / tiles, (N + wsn::kTile - 1) / wsn::kTile));
  }

  static int wgrad_chunks(int M, int Kr, int N, int* chunk) {
    int chunks = wgrad_chunk_bound(M, Kr, N);
    int c = (N + chunks - 1) / chunks;
    c = (c + wsn::kTk - 1) / wsn::kTk * wsn::kTk;
    chunks = (N + c - 1) / c;
    *chunk = c;
    return chunks;
  }

  ws_status setup(const ws_config& c, hipStream_t s) {
    cfg = c;
    stream = s;
    layers = layer_specs(c);
    n_params = total_params(layers);
    Lpos = c.window / c.patch;
    const int64_t nb = c.max_batch;
    const size_t pos = size_t(nb) * Lpos;
    hipError_t e = hipSuccess;
    auto A_ = [&](float** p, size_t floats) {
      if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(p), floats * sizeof(float), allocs);
    };
    A_(&theta, n_params);
    A_(&grad, n_params);
    A_(&adam_m, n_params);
    A_(&adam_v, n_params);
    A_(&mu, c.nx);
    A_(&sigma, c.nx);
    A_(&xb, size_t(2 * c.ny) * nb * c.window);
    A_(&tb, size_t(c.patch) * c.nx * pos);
    A_(&out, size_t(c.patch) * c.nx * pos);
    A_(&dout, size_t(c.patch) * c.nx * pos);
    H.assign(c.hidden + 1, nullptr);
    A.assign(c.hidden + 1, nullptr);
    for (int l = 0; l <= c.hidden; ++l) A_(&H[l], size_t(c.width) * pos);
    for (int l = 1; l <= c.hidden; ++l) A_(&A[l], size_t(c.width) * pos);
    for (int i = 0; i < 2; ++i) {
      A_(&dh[i], size_t(c.width) * pos);
      A_(&dz[i], size_t(c.width) * pos);
    }
    for (const auto& L : layers) {
      const int Kr = L.cin * L.K;
      part_floats = std::max<int64_t>(part_floats, int64_t(wgrad_chunk_bound(L.cout, Kr, int(pos))) * L.cout * (Kr + 1));
    }
    A_(&part, part_floats);
    A_(&loss_part, 1024);
    A_(&loss, 1);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&bad_index), sizeof(int), allocs);
    res_fast = (c.width == 128 || c.width == 256) && wsn::kResP % Lpos == 0 && c.hidden > 0;
    if (res_fast && e == hipSuccess)
      e = alloc(reinterpret_cast<void**>(&wt16), sizeof(short) * 3 * size_t(c.width) * c.width * c.hidden, allocs);
    if (e != hipSuccess)
      return fail(e == hipErrorOutOfMemory ? WS_ENOMEM : WS_EDEVICE, hip_msg(e, "device allocation"));
    std::vector<float> ones(c.nx, 1.f);
    e = hipMemsetAsync(theta, 0, sizeof(float) * n_params, stream);
    if (e == hipSuccess) e = hipMemsetAsync(adam_m, 0, sizeof(float) * n_params, stream);
    if (e == hipSuccess) e = hipMemsetAsync(adam_v, 0, sizeof(float) * n_params, stream);
    if (e == hipSuccess) e = hipMemsetAsync(mu, 0, sizeof(float) * c.nx, stream);
    if (e == hipSuccess) e = hipMemsetAsync(bad_index, 0, sizeof(int), stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sigma, ones.data(), sizeof(float) * c.nx, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(WS_EDEVICE, hip_msg(e, "initialisation"));
    return WS_OK;
  }

  template <int EPI>
  void conv(const wsn::ConvArgs& a, bool mfma = false) {
    const dim3 grid(unsigned((a.N + wsn::kTile - 1) / wsn::kTile), unsigned((a.M + wsn::kTile - 1) / wsn::kTile));
    if constexpr (EPI != wsn::kEpiBackward) {
      if (mfma) {
        hipLaunchKernelGGL(wsn::k_conv_mfma<EPI>, grid, dim3(wsn::kThreads), 0, stream, a);
        return;
      }
    }
    hipLaunchKernelGGL(wsn::k_conv<EPI>, grid, dim3(wsn::kThreads), 0, stream, a);
  }

  wsn::Gather gather_of(const LayerSpec& L, const float* src, int n, bool transpose_taps) const {
    const int W = cfg.window;
    if (&L == &layers.front()) return {src, n * W, L.K, Lpos, W, L.stride, L.dil, L.pad};
    if (transpose_taps) return {src, n * Lpos, L.K, Lpos, Lpos, 1, -L.dil, -L.pad};
    return {src, n * Lpos, L.K, Lpos, Lpos, 1, L.dil, L.pad};
  }

  // xb [2 ny][n W] -> out [P nx][n L]; keeps every activation for the backward pass
  // mfma: the inference form of the products (BF16 operands on the matrix
  // cores, FP32 accumulation); training always runs the FP32 kernels
  void forward(int n, bool mfma = false) {
    const int N = n * Lpos;
    const int Hn = cfg.hidden;
    {
      const LayerSpec& L = layers[0];
      wsn::ConvArgs a{L.cout, L.cin * L.K, N, theta + L.w_off, 0, theta + L.b_off, gather_of(L, xb, n, false),
                      H[0], nullptr, nullptr, nullptr};
      conv<wsn::kEpiRelu>(a, mfma);
    }
    for (int l = 1; l <= Hn; ++l) {
      const LayerSpec& L = layers[l];
      if (mfma && res_fast) {
        // the packed weights come from pack_residual(), run before the batch loop
        const wsn::ResidualArgs r{N, Lpos, L.dil, wt16 + size_t(l - 1) * 3 * L.cout * L.cout, theta + L.b_off,
                                  H[l - 1], H[l]};
        const dim3 grid(unsigned((N + wsn::kResP - 1) / wsn::kResP));
        if (L.cout == 128) hipLaunchKernelGGL(wsn::k_residual_mfma<128>, grid, dim3(256), 0, stream, r);
        else hipLaunchKernelGGL(wsn::k_residual_mfma<256>, grid, dim3(256), 0, stream, r);
        continue;
      }
      wsn::ConvArgs a{L.cout, L.cin * L.K, N, theta + L.w_off, 0, theta + L.b_off, gather_of(L, H[l - 1], n, false),
                      A[l], H[l], H[l - 1], nullptr};
      conv<wsn::kEpiResidual>(a, mfma);
    }
    const LayerSpec& L = layers[Hn + 1];
    wsn::ConvArgs a{L.cout, L.cin * L.K, N, theta + L.w_off, 0, theta + L.b_off, gather_of(L, H[Hn], n, false),
                    out, nullptr, nullptr, nullptr};
    conv<wsn::kEpiLinear>(a, mfma);
  }

  // BF16 tap-major copies of the residual weights for k_residual_mfma
  void pack_residual() {
    for (int l = 1; l <= cfg.hidden; ++l) {
      const LayerSpec& L = layers[l];
      const int64_t cnt = int64_t(3) * L.cout * L.cout;
      hipLaunchKernelGGL(wsn::k_pack_residual, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, stream,
                         static_cast<const float*>(theta + L.w_off), L.cout, wt16 + size_t(l - 1) * cnt);
    }
  }

  void wgrad(const LayerSpec& L, const float* D, const wsn::Gather& g, int N) {
    int chunk;
    const int Kr = L.cin * L.K;
    const int chunks = wgrad_chunks(L.cout, Kr, N, &chunk);
    const wsn::WgradArgs a{L.cout, Kr, N, chunk, D, g, part};
    const dim3 grid(unsigned((Kr + 1 + wsn::kTile - 1) / wsn::kTile), unsigned((L.cout + wsn::kTile - 1) / wsn::kTile),
                    unsigned(chunks));
    hipLaunchKernelGGL(wsn::k_wgrad, grid, dim3(wsn::kThreads), 0, stream, a);
    const int cnt = L.cout * (Kr + 1);
    hipLaunchKernelGGL(wsn::k_wgrad_reduce, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, stream,
                       static_cast<const float*>(part), chunks, L.cout, Kr, grad, L.w_off, L.b_off);
  }

  // loss of out against tb, gradient of every parameter into grad
  void loss_and_backward(int n) {
    const int N = n * Lpos;
    const int Hn = cfg.hidden;
    const int64_t count = int64_t(cfg.patch) * cfg.nx * N;
    const int blocks = int(std::min<int64_t>(1024, (count + 255) / 256));
    hipLaunchKernelGGL(wsn::k_mse, dim3(blocks), dim3(256), 0, stream, static_cast<const float*>(out),
                       static_cast<const float*>(tb), dout, count, float(2.0 / double(count)), loss_part);
    hipLaunchKernelGGL(wsn::k_sum, dim3(1), dim3(256), 0, stream, static_cast<const float*>(loss_part), blocks,
                       float(1.0 / double(count)), loss);
    const LayerSpec& LH = layers[Hn + 1];
    wgrad(LH, dout, gather_of(LH, H[Hn], n, false), N);
    {
      wsn::ConvArgs a{LH.cin, LH.cout * LH.K, N, theta + LH.w_off, 1, nullptr, gather_of(LH, dout, n, true),
                      dh[0], dz[0], nullptr, Hn >= 1 ? A[Hn] : H[0]};
      conv<wsn::kEpiBackward>(a);
    }
    int cur = 0;
    for (int l = Hn; l >= 1; --l) {
      const LayerSpec& L = layers[l];
      wgrad(L, dz[cur], gather_of(L, H[l - 1], n, false), N);
      wsn::ConvArgs a{L.cin, L.cout * L.K, N, theta + L.w_off, 1, nullptr, gather_of(L, dz[cur], n, true),
                      l > 1 ? dh[1 - cur] : nullptr, dz[1 - cur], dh[cur], l - 1 >= 1 ? A[l - 1] : H[0]};
      conv<wsn::kEpiBackward>(a);
      cur ^= 1;
    }
    const LayerSpec& L0 = layers[0];
    wgrad(L0, dz[cur], gather_of(L0, xb, n, false), N);
  }

  void gather_batch(const float* x, const float* lab, int64_t n_data, const int32_t* idx, int n) {
    const int64_t cnt = int64_t(n) * cfg.window;
    hipLaunchKernelGGL(wsn::k_gather_batch, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, stream, x, lab, n_data,
                       idx, n, 2 * cfg.ny, cfg.window, cfg.patch, cfg.nx, static_cast<const float*>(mu),
                       static_cast<const float*>(sigma), xb, lab ? tb : nullptr, bad_index);
  }

  // Waits for the stream; reports (and clears) an out-of-range batch index
  // seen since the last check.
  ws_status sync_and_check(const char* what) {
    int bad = 0;
    hipError_t e = hipMemcpyAsync(&bad, bad_index, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(WS_EDEVICE, hip_msg(e, what));
    if (bad) {
      e = hipMemsetAsync(bad_index, 0, sizeof(int), stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      return fail(WS_EINVAL, "a batch index was outside [0, n_data): its window was read as zeros");
    }
    return WS_OK;
  }
};

namespace {

ws_status launch_status(ws_t h, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return h->fail(WS_EDEVICE, hip_msg(e, what));
  return WS_OK;
}

const char* check_batch(ws_t h, const void* x, int64_t n_data, const int32_t* idx, int32_t n, bool limited) {
  if (!x || !idx) return "null device pointer";
  if (n_data < 1) return "n_data must be >= 1";
  if (n < 1) return "batch size must be >= 1";
  if (limited && n > h->cfg.max_batch) return "batch size exceeds max_batch";
  return nullptr;
}

}  // namespace

extern "C" {

void ws_config_defaults(ws_config* c) {
  if (!c) return;
  c->window = 64;
  c->patch = 4;
  c->width = 128;
  c->hidden = 4;
  c->nx = 5;
  c->ny = 2;
  c->max_batch = 1024;
}

int64_t ws_param_count(const ws_config* c) {
  if (!c || check_config(*c)) return 0;
  return total_params(layer_specs(*c));
}

ws_status ws_create(const ws_config* cfg, void* hip_stream, ws_t* out) {
  if (!out) {
    g_create_error = "out is NULL";
    return WS_EINVAL;
  }
  *out = nullptr;
  if (!cfg) {
    g_create_error = "cfg is NULL";
    return WS_EINVAL;
  }
  if (const char* m = check_config(*cfg)) {
    g_create_error = m;
    return WS_EINVAL;
  }
  ws_net* h = new (std::nothrow) ws_net();
  if (!h) {
    g_create_error = "host allocation failed";
    return WS_ENOMEM;
  }
  const ws_status s = h->setup(*cfg, static_cast<hipStream_t>(hip_stream));
  if (s != WS_OK) {
    g_create_error = h->err;
    delete h;
    return s;
  }
  *out = h;
  return WS_OK;
}

ws_status ws_set_params(ws_t h, const float* params, int64_t n) {
  if (!h) return WS_ESTATE;
  if (!params || n != h->n_params) return h->fail(WS_EINVAL, "params must hold ws_param_count() floats");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return h->fail(WS_EINVAL, "params must be finite");
  hipError_t e = hipMemcpyAsync(h->theta, params, sizeof(float) * n, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->adam_m, 0, sizeof(float) * n, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->adam_v, 0, sizeof(float) * n, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->fail(WS_EDEVICE, hip_msg(e, "parameter upload"));
  h->step = 0;
  return WS_OK;
}

ws_status ws_get_params(ws_t h, float* params, int64_t n) {
  if (!h) return WS_ESTATE;
  if (!params || n != h->n_params) return h->fail(WS_EINVAL, "params must hold ws_param_count() floats");
  hipError_t e = hipMemcpyAsync(params, h->theta, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->fail(WS_EDEVICE, hip_msg(e, "parameter download"));
  return WS_OK;
}

ws_status ws_set_normalization(ws_t h, const float* mu, const float* sigma) {
  if (!h) return WS_ESTATE;
  if (!mu || !sigma) return h->fail(WS_EINVAL, "mu and sigma are required");
  for (int i = 0; i < h->cfg.nx; ++i)
    if (!std::isfinite(mu[i]) || !std::isfinite(sigma[i]) || !(sigma[i] > 0.f))
      return h->fail(WS_EINVAL, "mu must be finite and sigma finite and positive");
  hipError_t e = hipMemcpyAsync(h->mu, mu, sizeof(float) * h->cfg.nx, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->sigma, sigma, sizeof(float) * h->cfg.nx, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->fail(WS_EDEVICE, hip_msg(e, "normalisation upload"));
  return WS_OK;
}

ws_status ws_set_tracks(ws_t h, const int64_t* offsets, int32_t n_tracks, int64_t* n_windows) {
  if (!h) return WS_ESTATE;
  if (!offsets || n_tracks < 1) return h->fail(WS_EINVAL, "offsets and n_tracks >= 1 are required");
  if (offsets[0] != 0) return h->fail(WS_EINVAL, "offsets[0] must be 0");
  const int W = h->cfg.window;
  std::vector<int> track, start, first(size_t(n_tracks) + 1, 0);
  for (int i = 0; i < n_tracks; ++i) {
    const int64_t T = offsets[i + 1] - offsets[i];
    if (T < 1) return h->fail(WS_EINVAL, "every track needs T >= 1 measurements");
    if (T > (int64_t(1) << 30)) return h->fail(WS_EINVAL, "track too long");
    const int64_t nw = (T + W - 1) / W;
    if (int64_t(track.size()) + nw > (int64_t(1) << 31) - 1) return h->fail(WS_EINVAL, "too many windows");
    for (int64_t w = 0; w < nw; ++w) {
      track.push_back(i);
      start.push_back(int(w < nw - 1 ? 1 + W * w : std::max<int64_t>(1, T - W + 1)));
    }
    first[i + 1] = int(track.size());
  }
  for (void* p : h->plan_allocs) (void)hipFree(p);
  h->plan_allocs.clear();
  h->n_windows = 0;
  h->n_tracks = 0;
  const size_t nw = track.size();
  hipError_t e = h->alloc(reinterpret_cast<void**>(&h->win_track), sizeof(int) * nw, h->plan_allocs);
  if (e == hipSuccess) e = h->alloc(reinterpret_cast<void**>(&h->win_start), sizeof(int) * nw, h->plan_allocs);
  if (e == hipSuccess) e = h->alloc(reinterpret_cast<void**>(&h->first), sizeof(int) * first.size(), h->plan_allocs);
  if (e == hipSuccess)
    e = h->alloc(reinterpret_cast<void**>(&h->meas_off), sizeof(int64_t) * (size_t(n_tracks) + 1), h->plan_allocs);
  if (e == hipSuccess) e = hipMemcpyAsync(h->win_track, track.data(), sizeof(int) * nw, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->win_start, start.data(), sizeof(int) * nw, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->meas_off, offsets, sizeof(int64_t) * (size_t(n_tracks) + 1), hipMemcpyHostToDevice,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->fail(e == hipErrorOutOfMemory ? WS_ENOMEM : WS_EDEVICE, hip_msg(e, "window plan"));
  h->n_windows = int64_t(nw);
  h->n_tracks = n_tracks;
  if (n_windows) *n_windows = int64_t(nw);
  return WS_OK;
}

ws_status ws_windows(ws_t h, const double* d_y, float* d_x) {
  if (!h) return WS_ESTATE;
  if (!h->n_windows) return h->fail(WS_ESTATE, "no tracks planned (ws_set_tracks)");
  if (!d_y || !d_x) return h->fail(WS_EINVAL, "null device pointer");
  if (h->n_windows > (int64_t(1) << 31) - 1) return h->fail(WS_EINVAL, "too many windows");
  const int64_t cnt = h->n_windows * h->cfg.window;
  hipLaunchKernelGGL(wsn::k_features, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, h->stream, h->table(), d_y,
                     h->cfg.ny, h->cfg.window, int64_t(0), int(h->n_windows), 0, d_x);
  return launch_status(h, "feature kernel");
}

ws_status ws_labels(ws_t h, const double* d_mean, float* d_lab) {
  if (!h) return WS_ESTATE;
  if (!h->n_windows) return h->fail(WS_ESTATE, "no tracks planned (ws_set_tracks)");
  if (!d_mean || !d_lab) return h->fail(WS_EINVAL, "null device pointer");
  const int64_t cnt = h->n_windows * h->cfg.window;
  hipLaunchKernelGGL(wsn::k_labels, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, h->stream, h->table(), d_mean,
                     h->cfg.nx, h->cfg.window, h->n_windows, d_lab);
  return launch_status(h, "label kernel");
}

ws_status ws_train_step(ws_t h, const float* d_x, const float* d_lab, int64_t n_data, const int32_t* d_idx,
                        int32_t n, const ws_adam* opt, float* loss_out) {
  if (!h) return WS_ESTATE;
  if (const char* m = check_batch(h, d_x, n_data, d_idx, n, true)) return h->fail(WS_EINVAL, m);
  if (!d_lab || !opt) return h->fail(WS_EINVAL, "labels and optimiser settings are required");
  if (!(opt->lr > 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) || !(opt->beta2 >= 0.f && opt->beta2 < 1.f) ||
      !(opt->eps > 0.f))
    return h->fail(WS_EINVAL, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
  h->gather_batch(d_x, d_lab, n_data, d_idx, n);
  h->forward(n);
  h->loss_and_backward(n);
  h->step += 1;
  const float c1 = float(1.0 - std::pow(double(opt->beta1), double(h->step)));
  const float c2 = float(1.0 - std::pow(double(opt->beta2), double(h->step)));
  hipLaunchKernelGGL(wsn::k_adam, dim3(unsigned((h->n_params + 255) / 256)), dim3(256), 0, h->stream, h->theta,
                     static_cast<const float*>(h->grad), h->adam_m, h->adam_v, h->n_params, opt->lr, opt->beta1,
                     opt->beta2, opt->eps, c1, c2);
  ws_status s = launch_status(h, "training step");
  if (s != WS_OK || !loss_out) return s;
  const hipError_t e = hipMemcpyAsync(loss_out, h->loss, sizeof(float), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return h->fail(WS_EDEVICE, hip_msg(e, "loss download"));
  return h->sync_and_check("loss download");
}

ws_status ws_gradient(ws_t h, const float* d_x, const float* d_lab, int64_t n_data, const int32_t* d_idx,
                      int32_t n, float* grad, float* loss_out) {
  if (!h) return WS_ESTATE;
  if (const char* m = check_batch(h, d_x, n_data, d_idx, n, true)) return h->fail(WS_EINVAL, m);
  if (!d_lab) return h->fail(WS_EINVAL, "labels are required");
  h->gather_batch(d_x, d_lab, n_data, d_idx, n);
  h->forward(n);
  h->loss_and_backward(n);
  ws_status s = launch_status(h, "gradient");
  if (s != WS_OK) return s;
  hipError_t e = hipSuccess;
  if (grad) e = hipMemcpyAsync(grad, h->grad, sizeof(float) * h->n_params, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && loss_out) e = hipMemcpyAsync(loss_out, h->loss, sizeof(float), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return h->fail(WS_EDEVICE, hip_msg(e, "gradient download"));
  return h->sync_and_check("gradient download");
}

ws_status ws_predict(ws_t h, const float* d_x, int64_t n_data, const int32_t* d_idx, int32_t n, float* d_states) {
  if (!h) return WS_ESTATE;
  if (const char* m = check_batch(h, d_x, n_data, d_idx, n, false)) return h->fail(WS_EINVAL, m);
  if (!d_states) return h->fail(WS_EINVAL, "null device pointer");
  const int W = h->cfg.window;
  for (int32_t b0 = 0; b0 < n; b0 += h->cfg.max_batch) {
    const int nb = std::min(h->cfg.max_batch, n - b0);
    h->gather_batch(d_x, nullptr, n_data, d_idx + b0, nb);
    h->forward(nb);
    const int64_t cnt = int64_t(nb) * W;
    hipLaunchKernelGGL(wsn::k_states, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, h->stream,
                       static_cast<const float*>(h->out), nb, W, h->cfg.patch, h->cfg.nx,
                       static_cast<const float*>(h->mu), static_cast<const float*>(h->sigma),
                       d_states + size_t(b0) * W * h->cfg.nx);
  }
  const ws_status s = launch_status(h, "prediction");
  if (s != WS_OK) return s;
  return h->sync_and_check("prediction");
}

static ws_status trajectory(ws_t h, const double* d_y, double* d_mean, bool mfma) {
  if (!h) return WS_ESTATE;
  if (!h->n_windows) return h->fail(WS_ESTATE, "no tracks planned (ws_set_tracks)");
  if (!d_y || !d_mean) return h->fail(WS_EINVAL, "null device pointer");
  const int W = h->cfg.window;
  if (mfma && h->res_fast) h->pack_residual();
  for (int64_t w0 = 0; w0 < h->n_windows; w0 += h->cfg.max_batch) {
    const int nb = int(std::min<int64_t>(h->cfg.max_batch, h->n_windows - w0));
    const int64_t cnt = int64_t(nb) * W;
    const dim3 grid(unsigned((cnt + 255) / 256));
    hipLaunchKernelGGL(wsn::k_features, grid, dim3(256), 0, h->stream, h->table(), d_y, h->cfg.ny, W, w0, nb, 1,
                       h->xb);
    h->forward(nb, mfma);
    hipLaunchKernelGGL(wsn::k_scatter, grid, dim3(256), 0, h->stream, h->table(), static_cast<const float*>(h->out),
                       w0, nb, W, h->cfg.patch, h->cfg.nx, static_cast<const float*>(h->mu),
                       static_cast<const float*>(h->sigma), d_mean);
  }
  return launch_status(h, "trajectory");
}

ws_status ws_trajectory(ws_t h, const double* d_y, double* d_mean) { return trajectory(h, d_y, d_mean, false); }

ws_status ws_trajectory_mfma(ws_t h, const double* d_y, double* d_mean) { return trajectory(h, d_y, d_mean, true); }

const char* ws_last_error(ws_t h) { return h ? h->err.c_str() : g_create_error.c_str(); }

void ws_destroy(ws_t h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

}  // extern "C"
