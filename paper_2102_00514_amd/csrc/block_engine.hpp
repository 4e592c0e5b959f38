// Stacked coordinated-turn targets that do not interact, smoothed by the
// iterated extended (Taylor) smoother as separate blocks.
//
// With k targets stacked in one state (nx = 5k), block-diagonal Q, P0 and
// initial covariances, and every sensor measuring one target with no noise
// correlation between sensors of different targets, the first-order Taylor
// linearisation (eq. 10) of f and h is block-diagonal: F and H act block by
// block and Lambda = Omega = 0.  The filter and smoother of every iteration
// then keep block-diagonal covariances, and the iterated smoother of the
// stacked problem is the k smoothers of the blocks, exact up to rounding.
// Each block runs on its own engine and the results are reassembled.
//
// Sigma-point linearisation (eq. 7-9) does not separate: sigma points that
// move one target also shift the regression means of the others, so the
// residual covariances gain terms between targets (-d_b d_c^T, d_b = g_b(xbar)
// - zbar_b); stacked problems with those rules are not accepted here.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "engine_base.hpp"

namespace pks {

using EngineFactory = EngineBase* (*)(int model, int precision, int nx, int ny);

class BlockEngine final : public EngineBase {
 public:
  static constexpr int kB = 5;  // states per coordinated-turn block

  explicit BlockEngine(EngineFactory make) : make_(make) {}

  sm_status setup(const sm_problem& pb, hipStream_t st) override {
    stream = st;
    N_ = pb.nx;
    k_ = pb.nx / kB;
    P_ = pb.ny;
    ntracks = pb.n_tracks;
    n_iter = pb.n_iter;
    S = pb.offsets[pb.n_tracks] + pb.n_tracks;
    sensors_.assign(k_, {});
    for (int s = 0; s < P_; ++s) sensors_[int(pb.params[3 + 3 * s])].push_back(s);
    const int pb_ = P_ / k_;
    const int64_t nmeas = pb.offsets[pb.n_tracks];
    for (int b = 0; b < k_; ++b) {
      const int o = b * kB;
      std::vector<double> prm(1 + 3 * pb_), Q(kB * kB), R(pb_ * pb_), m0(size_t(ntracks) * kB),
          P0(size_t(ntracks) * kB * kB), y(size_t(nmeas) * pb_), im, ic;
      prm[0] = pb.params[0];
      for (int s = 0; s < pb_; ++s) {
        const int g = sensors_[b][s];
        prm[1 + 3 * s] = pb.params[1 + 3 * g];
        prm[2 + 3 * s] = pb.params[2 + 3 * g];
        prm[3 + 3 * s] = 0.0;
        for (int t = 0; t < pb_; ++t) R[s * pb_ + t] = pb.R[g * P_ + sensors_[b][t]];
      }
      for (int i = 0; i < kB; ++i)
        for (int j = 0; j < kB; ++j) Q[i * kB + j] = pb.Q[(o + i) * N_ + o + j];
      for (int t = 0; t < ntracks; ++t) {
        for (int i = 0; i < kB; ++i) {
          m0[size_t(t) * kB + i] = pb.m0[size_t(t) * N_ + o + i];
          for (int j = 0; j < kB; ++j)
            P0[(size_t(t) * kB + i) * kB + j] = pb.P0[(size_t(t) * N_ + o + i) * N_ + o + j];
        }
      }
      for (int64_t r = 0; r < nmeas; ++r)
        for (int s = 0; s < pb_; ++s) y[size_t(r) * pb_ + s] = pb.y[size_t(r) * P_ + sensors_[b][s]];
      sm_problem q = pb;
      q.nx = kB;
      q.ny = pb_;
      q.params = prm.data();
      q.n_params = int(prm.size());
      q.Q = Q.data();
      q.R = R.data();
      q.m0 = m0.data();
      q.P0 = P0.data();
      q.y = y.data();
      if (pb.init_mean) {
        im.resize(size_t(S) * kB);
        for (int64_t s = 0; s < S; ++s)
          for (int i = 0; i < kB; ++i) im[size_t(s) * kB + i] = pb.init_mean[size_t(s) * N_ + o + i];
        q.init_mean = im.data();
      }
      if (pb.init_cov) {
        ic.resize(size_t(S) * kB * kB);
        for (int64_t s = 0; s < S; ++s)
          for (int i = 0; i < kB; ++i)
            for (int j = 0; j < kB; ++j)
              ic[(size_t(s) * kB + i) * kB + j] = pb.init_cov[(size_t(s) * N_ + o + i) * N_ + o + j];
        q.init_cov = ic.data();
      }
      q.max_device_bytes = pb.max_device_bytes > 0 ? std::max<int64_t>(1, pb.max_device_bytes / k_) : 0;
      std::unique_ptr<EngineBase> e(make_(q.model, q.precision, q.nx, q.ny));
      if (!e) return fail(SM_EINVAL, "no kernel for the blocks of this configuration");
      const sm_status s = e->setup(q, stream);
      if (s != SM_OK) return fail(s, "block " + std::to_string(b) + ": " + e->err);
      device_bytes += e->device_bytes;
      blocks_.push_back(std::move(e));
    }
    sched_lanes = blocks_[0]->sched_lanes;
    sched_slots = blocks_[0]->sched_slots;
    sched_tiles = blocks_[0]->sched_tiles;
    return SM_OK;
  }

  sm_status iterate(int k) override {
    for (auto& b : blocks_) {
      const sm_status s = b->iterate(k);
      if (s != SM_OK) return fail(s, b->err);
    }
    iters += k;
    return SM_OK;
  }

  // Per track, the largest change over the blocks (NaN if any block's is NaN).
  sm_status track_deltas(double* out) override {
    std::vector<double> d(ntracks + 1);
    for (int i = 0; i <= ntracks; ++i) out[i] = 0.0;
    for (auto& b : blocks_) {
      const sm_status s = b->track_deltas(d.data());
      if (s != SM_OK) return fail(s, b->err);
      for (int i = 0; i <= ntracks; ++i) out[i] = (d[i] > out[i] || d[i] != d[i]) ? d[i] : out[i];
    }
    return SM_OK;
  }

  sm_status result_host(double* mean, double* cov) override {
    std::vector<double> m(mean ? size_t(S) * kB : 0), c(cov ? size_t(S) * kB * kB : 0);
    if (cov) std::fill(cov, cov + size_t(S) * N_ * N_, 0.0);
    for (int b = 0; b < k_; ++b) {
      const sm_status s = blocks_[b]->result_host(mean ? m.data() : nullptr, cov ? c.data() : nullptr);
      if (s != SM_OK) return fail(s, blocks_[b]->err);
      const int o = b * kB;
      for (int64_t sl = 0; sl < S; ++sl)
        for (int i = 0; i < kB; ++i) {
          if (mean) mean[size_t(sl) * N_ + o + i] = m[size_t(sl) * kB + i];
          if (cov)
            for (int j = 0; j < kB; ++j)
              cov[(size_t(sl) * N_ + o + i) * N_ + o + j] = c[(size_t(sl) * kB + i) * kB + j];
        }
    }
    return SM_OK;
  }

  sm_status result_device(void* mean, void* cov) override {
    if (cov) {
      const size_t word = precision_word();
      const hipError_t e = hipMemsetAsync(cov, 0, word * size_t(S) * N_ * N_, stream);
      if (e != hipSuccess) return fail(SM_EDEVICE, hip_msg(e, "clearing the covariance output"));
    }
    for (int b = 0; b < k_; ++b) {
      const sm_status s = blocks_[b]->result_device_placed(mean, cov, N_, b * kB);
      if (s != SM_OK) return fail(s, blocks_[b]->err);
    }
    return SM_OK;
  }

  sm_status set_trajectory_device(const void* mean, const void* cov, const double* cov_const) override {
    std::vector<double> cb(kB * kB);
    for (int b = 0; b < k_; ++b) {
      const int o = b * kB;
      if (cov_const)
        for (int i = 0; i < kB; ++i)
          for (int j = 0; j < kB; ++j) cb[i * kB + j] = cov_const[(o + i) * N_ + o + j];
      const sm_status s = blocks_[b]->set_trajectory_placed(mean, cov, cov_const ? cb.data() : nullptr, N_, o);
      if (s != SM_OK) return fail(s, blocks_[b]->err);
    }
    iters = 0;
    return SM_OK;
  }

  sm_status profile(int k, int repeat, sm_kernel_time* out, int cap_out, int* n_out) override {
    std::vector<sm_kernel_time> acc;
    std::vector<sm_kernel_time> one(64);
    for (auto& b : blocks_) {
      int n = 0;
      const sm_status s = b->profile(k, repeat, one.data(), int(one.size()), &n);
      if (s != SM_OK) return fail(s, b->err);
      for (int i = 0; i < n; ++i) {
        auto it = std::find_if(acc.begin(), acc.end(),
                               [&](const sm_kernel_time& t) { return std::strcmp(t.name, one[i].name) == 0; });
        if (it == acc.end()) {
          acc.push_back(one[i]);
        } else {
          it->launches += one[i].launches;
          it->total_ms += one[i].total_ms;
          it->positions += one[i].positions;
        }
      }
    }
    iters += k;
    const int n = std::min<int>(cap_out, int(acc.size()));
    for (int i = 0; i < n; ++i) out[i] = acc[i];
    if (n_out) *n_out = n;
    return SM_OK;
  }

  // The objective of the stacked state is the sum of the blocks' objectives;
  // one damping value per track acts on every block (I/lambda is
  // block-diagonal), so the blocks take or reject their steps together.
  sm_status objective(double* out) override {
    std::vector<double> c(ntracks);
    std::fill(out, out + ntracks, 0.0);
    for (auto& b : blocks_) {
      const sm_status s = b->objective(c.data());
      if (s != SM_OK) return fail(s, b->err);
      for (int i = 0; i < ntracks; ++i) out[i] += c[i];
    }
    return SM_OK;
  }

  // Independent targets: the filtered moments are block-diagonal and the log
  // likelihood of the stacked measurements is the sum over the blocks.
  sm_status filter(double* mean, double* cov, double* loglik) override {
    std::vector<double> m(mean ? size_t(S) * kB : 0), c(cov ? size_t(S) * kB * kB : 0), l(ntracks);
    if (cov) std::fill(cov, cov + size_t(S) * N_ * N_, 0.0);
    if (loglik) std::fill(loglik, loglik + ntracks, 0.0);
    for (int b = 0; b < k_; ++b) {
      const sm_status s = blocks_[b]->filter(mean ? m.data() : nullptr, cov ? c.data() : nullptr, l.data());
      if (s != SM_OK) return fail(s, blocks_[b]->err);
      if (loglik)
        for (int i = 0; i < ntracks; ++i) loglik[i] += l[i];
      const int o = b * kB;
      for (int64_t sl = 0; sl < S; ++sl)
        for (int i = 0; i < kB; ++i) {
          if (mean) mean[size_t(sl) * N_ + o + i] = m[size_t(sl) * kB + i];
          if (cov)
            for (int j = 0; j < kB; ++j)
              cov[(size_t(sl) * N_ + o + i) * N_ + o + j] = c[(size_t(sl) * kB + i) * kB + j];
        }
    }
    return SM_OK;
  }

  sm_status lm_mode(bool on) override { return each([&](EngineBase& b) { return b.lm_mode(on); }); }
  sm_status lm_set_lambda(const double* lam) override {
    return each([&](EngineBase& b) { return b.lm_set_lambda(lam); });
  }
  sm_status lm_save() override { return each([](EngineBase& b) { return b.lm_save(); }); }
  sm_status lm_restore(const unsigned char* reject) override {
    return each([&](EngineBase& b) { return b.lm_restore(reject); });
  }

  void set_precision_word(size_t w) { word_ = w; }

 private:
  template <class F>
  sm_status each(F&& f) {
    for (auto& b : blocks_) {
      const sm_status s = f(*b);
      if (s != SM_OK) return fail(s, b->err);
    }
    return SM_OK;
  }

  size_t precision_word() const { return word_; }

  EngineFactory make_;
  int N_ = 0, k_ = 0, P_ = 0;
  size_t word_ = sizeof(double);
  std::vector<std::vector<int>> sensors_;
  std::vector<std::unique_ptr<EngineBase>> blocks_;
};

}  // namespace pks
