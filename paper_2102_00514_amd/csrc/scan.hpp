// Device-wide inclusive scan with an expensive associative operator.
//
// Scan positions 0..m-1 are cut into tiles of B lanes x K positions.  Each lane
// folds its K consecutive elements sequentially; the B lane aggregates of a
// tile are scanned in LDS by a Kogge-Stone ladder (log2 B combine steps, all
// lanes busy, entry-major LDS layout so that lane i touches word i of each row:
// no bank conflicts).  The up-sweep writes every lane's exclusive prefix and the
// tile aggregate; the tile aggregates are scanned recursively; the down-sweep
// then starts each lane from (tile carry) (x) (lane exclusive prefix) and walks
// its K elements with the cheap carry form of the operator, writing the
// inclusive prefix of every position.
//
// The first scan position always holds a carry-form element (a prior element
// for filtering, an end element for smoothing), so every prefix that starts at
// position 0 is a carry and no identity element is ever needed.
#pragma once

#include "linalg.hpp"

namespace pks {

struct ScanArgs {
  const void* elems;   // elements, [kElemWords][estride]
  size_t estride;
  int64_t m;           // number of scan positions
  int reverse;         // position q is stored at index m-1-q (level 0 only)
  int K;               // positions per lane
  void* lane_excl;     // [kElemWords][lstride], lane exclusive prefixes
  size_t lstride;
  void* tile_agg;      // [kElemWords][tstride], tile aggregates (scan order)
  size_t tstride;
  const void* tile_carry;  // [kCarryWords][cstride], inclusive carries of the tiles
  size_t cstride;
  void* out;           // [kCarryWords][ostride], inclusive carry of every position
  size_t ostride;
};

// Inclusive scan of the B lane values of a block.  Scan position q = lane
// (FWD) or B-1-lane (reverse).  Inside a wavefront the Kogge-Stone steps move
// elements with cross-lane shuffles (no LDS, no barriers); across wavefronts
// (B > 64) only each wavefront's total goes through LDS: lds holds B/64
// elements, entry-major with row stride B/64.  On exit v is the inclusive
// prefix at q and, when has_ex (q > 0), ex the exclusive one.  Invalid lanes
// must form a suffix of the scan order: no valid lane reads their values.  A
// wavefront whose lanes are all invalid passes active = false (wavefront-
// uniform): it skips its combines and only takes part in the barrier.
template <class Op, int B, bool FWD, typename R>
PKS_DEV void block_ladder(R* lds, typename Op::Elem& v, typename Op::Elem& ex, bool& has_ex, bool active = true) {
  constexpr int NW = B / 64;
  static_assert(B % 64 == 0, "whole wavefronts");
  const int pl = int(threadIdx.x), wl = pl & 63, w = pl >> 6;
  const int qw = FWD ? wl : 63 - wl;        // scan position inside the wavefront
  const int qwave = FWD ? w : NW - 1 - w;   // scan position of the wavefront
  if (active) {
    auto step = [&](int d) {
      typename Op::Elem left;
      const int src = FWD ? (wl >= d ? wl - d : wl) : (wl + d < 64 ? wl + d : wl);
      Op::shfl(v, src, left);
      if (qw >= d) {
        typename Op::Elem r;
        Op::combine(left, v, r);
        v = r;
      }
    };
    if constexpr (Op::kCompact) {
      // one copy of a long operator instead of six
#pragma unroll 1
      for (int d = 1; d < 64; d <<= 1) step(d);
    } else {
      PKS_UNROLL for (int d = 1; d < 64; d <<= 1) step(d);
    }
  }
  typename Op::Elem wp;   // total of the wavefronts before this one (qwave > 0)
  if constexpr (NW > 1) {
    if (active && qw == 63) Op::store(lds, NW, qwave, v);
    __syncthreads();
    if (active && qwave > 0) {
      Op::load(lds, NW, 0, wp);
      for (int k = 1; k < qwave; ++k) {
        typename Op::Elem t, r;
        Op::load(lds, NW, k, t);
        Op::combine(wp, t, r);
        wp = r;
      }
      typename Op::Elem r;
      Op::combine(wp, v, r);
      v = r;
    }
  }
  has_ex = false;
  if (!active) return;
  const int src = FWD ? (wl > 0 ? wl - 1 : wl) : (wl < 63 ? wl + 1 : wl);
  Op::shfl(v, src, ex);
  has_ex = qw > 0;
  if constexpr (NW > 1) {
    if (qw == 0 && qwave > 0) {
      ex = wp;
      has_ex = true;
    }
  }
}

template <class Op, int B, typename R>
__global__ __launch_bounds__(B) void k_scan_up(ScanArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  const R* E = static_cast<const R*>(a.elems);
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t first = (tile * B + lane) * a.K;
  const bool valid = first < a.m;
  typename Op::Elem v{};   // invalid lanes feed the ladder zeros
  if (valid) {
    const int64_t idx0 = a.reverse ? a.m - 1 - first : first;
    Op::load(E, a.estride, idx0, v);
    for (int j = 1; j < a.K; ++j) {
      const int64_t q = first + j;
      if (q >= a.m) break;
      typename Op::Elem e, r;
      Op::load(E, a.estride, a.reverse ? a.m - 1 - q : q, e);
      Op::combine(v, e, r);
      v = r;
    }
  }
  typename Op::Elem ex;
  bool has_ex;
  const bool wave_active = (tile * B + (lane & ~63)) * a.K < a.m;
  block_ladder<Op, B, true, R>(lds, v, ex, has_ex, wave_active);
  R* LX = static_cast<R*>(a.lane_excl);
  if (valid && has_ex) Op::store(LX, a.lstride, tile * B + lane, ex);
  // last valid lane of the tile publishes the tile aggregate
  const int64_t rem = a.m - tile * B * (int64_t)a.K;
  const int64_t nvalid = (rem + a.K - 1) / a.K;
  const int last = nvalid < B ? int(nvalid) - 1 : B - 1;
  if (lane == last) Op::store(static_cast<R*>(a.tile_agg), a.tstride, tile, v);
}

template <class Op, int B, typename R>
PKS_DEV void lane_apply(const ScanArgs& a, int64_t first, bool have, typename Op::Carry& c) {
  const R* E = static_cast<const R*>(a.elems);
  R* O = static_cast<R*>(a.out);
  for (int j = 0; j < a.K; ++j) {
    const int64_t q = first + j;
    if (q >= a.m) break;
    const int64_t idx = a.reverse ? a.m - 1 - q : q;
    typename Op::Elem e;
    Op::load(E, a.estride, idx, e);
    if (have) {
      typename Op::Carry n;
      Op::apply(c, e, n);
      c = n;
    } else {
      Op::to_carry(e, c);
      have = true;
    }
    Op::store(O, a.ostride, idx, c);
  }
}

template <class Op, int B, typename R>
__global__ __launch_bounds__(B) void k_scan_down(ScanArgs a) {
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t first = (tile * B + lane) * a.K;
  if (first >= a.m) return;
  typename Op::Carry c;
  bool have = false;
  if (tile > 0) {
    Op::load(static_cast<const R*>(a.tile_carry), a.cstride, tile - 1, c);
    have = true;
  }
  if (lane > 0) {
    typename Op::Elem ex;
    Op::load(static_cast<const R*>(a.lane_excl), a.lstride, tile * B + lane, ex);
    if (have) {
      typename Op::Carry n;
      Op::apply(c, ex, n);
      c = n;
    } else {
      Op::to_carry(ex, c);
      have = true;
    }
  }
  lane_apply<Op, B, R>(a, first, have, c);
}

// Whole inclusive scan of m positions by one block (K = ceil(m / B) per lane):
// fold, ladder, then every lane walks its positions from its exclusive carry.
template <class Op, int B, typename R>
PKS_DEV void block_scan(R* lds, int lane, const R* E, size_t estride, int64_t m, int reverse, R* out,
                        size_t ostride) {
  const int K = int((m + B - 1) / B);
  const int64_t first = (int64_t)lane * K;
  const bool valid = first < m;
  typename Op::Elem v{};   // invalid lanes feed the ladder zeros
  if (valid) {
    Op::load(E, estride, reverse ? m - 1 - first : first, v);
    for (int j = 1; j < K; ++j) {
      const int64_t q = first + j;
      if (q >= m) break;
      typename Op::Elem e, r;
      Op::load(E, estride, reverse ? m - 1 - q : q, e);
      Op::combine(v, e, r);
      v = r;
    }
  }
  typename Op::Elem ex;
  bool has_ex;
  block_ladder<Op, B, true, R>(lds, v, ex, has_ex, int64_t(lane & ~63) * K < m);
  if (!valid) return;
  if (K == 1) {
    // v is the inclusive prefix of this lane's position, and it starts at a
    // carry-form element, so its carry part is the result
    typename Op::Carry c;
    Op::to_carry(v, c);
    Op::store(out, ostride, reverse ? m - 1 - first : first, c);
    return;
  }
  typename Op::Carry c;
  bool have = false;
  if (has_ex) {
    Op::to_carry(ex, c);
    have = true;
  }
  for (int j = 0; j < K; ++j) {
    const int64_t q = first + j;
    if (q >= m) break;
    const int64_t idx = reverse ? m - 1 - q : q;
    typename Op::Elem e;
    Op::load(E, estride, idx, e);
    if (have) {
      typename Op::Carry n;
      Op::apply(c, e, n);
      c = n;
    } else {
      Op::to_carry(e, c);
      have = true;
    }
    Op::store(out, ostride, idx, c);
  }
}

// Whole scan in one block.
template <class Op, int B, typename R>
__global__ __launch_bounds__(B) void k_scan_single(ScanArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  block_scan<Op, B, R>(reinterpret_cast<R*>(smem_raw), threadIdx.x, static_cast<const R*>(a.elems), a.estride,
                       a.m, a.reverse, static_cast<R*>(a.out), a.ostride);
}

}  // namespace pks
