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

// Lane moves of the wavefront ladder.  An element crosses lanes as its words
// do, each 64-bit word as two 32-bit halves; DPP moves run on the VALU of the
// wavefront's own SIMD, where a shuffle through the LDS crossbar would share
// the compute unit's LDS bandwidth with the other wavefronts of the block.
template <int CTRL, int ROWMASK>
struct DppMove {
  // lanes without a source read 0 and lanes of rows outside ROWMASK keep an
  // undefined value: neither is ever combined
  PKS_DEV static int mv32(int x) { return __builtin_amdgcn_mov_dpp(x, CTRL, ROWMASK, 0xf, true); }
  PKS_DEV double operator()(double x) const {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(x));
    const unsigned lo = static_cast<unsigned>(mv32(static_cast<int>(static_cast<unsigned>(u))));
    const unsigned hi = static_cast<unsigned>(mv32(static_cast<int>(static_cast<unsigned>(u >> 32))));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
  }
  PKS_DEV float operator()(float x) const { return __int_as_float(mv32(__float_as_int(x))); }
};

// The value of lane hi_src in lanes of rows 2 and 3, of lane lo_src in rows 0
// and 1 (v_readlane: a wavefront-uniform read of one lane).
struct LanePick {
  int upper;   // this lane is in rows 2 or 3
  int lo_src, hi_src;
  PKS_DEV static int rd(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
  PKS_DEV float operator()(float x) const {
    const int xi = __float_as_int(x);
    const int a = rd(xi, lo_src), b = rd(xi, hi_src);
    return __int_as_float(upper ? b : a);
  }
  PKS_DEV double operator()(double x) const {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(x));
    const int lo = static_cast<int>(static_cast<unsigned>(u)), hi = static_cast<int>(static_cast<unsigned>(u >> 32));
    const unsigned a0 = static_cast<unsigned>(rd(lo, lo_src)), a1 = static_cast<unsigned>(rd(hi, lo_src));
    const unsigned b0 = static_cast<unsigned>(rd(lo, hi_src)), b1 = static_cast<unsigned>(rd(hi, hi_src));
    const unsigned long long r = upper ? ((static_cast<unsigned long long>(b1) << 32) | b0)
                                       : ((static_cast<unsigned long long>(a1) << 32) | a0);
    return __longlong_as_double(static_cast<long long>(r));
  }
};

// One Kogge-Stone step of the wavefront ladder: left = the element of the
// lane before this one at the step's distance, in scan order.  The wavefront
// is four rows of 16 lanes.  Steps 0-3 scan each row (distance 1, 2, 4, 8
// inside the row: DPP row shifts); step 4 hands the total of rows 0 and 2 to
// rows 1 and 3, step 5 the running total of rows 0-1 to rows 2 and 3 (forward:
// DPP row broadcasts; reverse, where rows run 3, 2, 1, 0: the totals of rows 3
// and 1 to rows 2 and 0, then rows 3-2 to rows 1 and 0, by lane reads).
// Returns whether this lane combines at the step.
template <class Op, bool FWD>
PKS_DEV bool ladder_step(int s, int wl, const typename Op::Elem& v, typename Op::Elem& left) {
  const int in_row = FWD ? (wl & 15) : 15 - (wl & 15);   // scan position inside the row
  const int row = wl >> 4;
  const int qrow = FWD ? row : 3 - row;                    // scan position of the row
  if constexpr (FWD) {
    switch (s) {
      case 0: Op::move(v, DppMove<0x111, 0xf>{}, left); break;   // row_shr:1
      case 1: Op::move(v, DppMove<0x112, 0xf>{}, left); break;   // row_shr:2
      case 2: Op::move(v, DppMove<0x114, 0xf>{}, left); break;   // row_shr:4
      case 3: Op::move(v, DppMove<0x118, 0xf>{}, left); break;   // row_shr:8
      case 4: Op::move(v, DppMove<0x142, 0xa>{}, left); break;   // row_bcast:15 into rows 1, 3
      default: Op::move(v, DppMove<0x143, 0xc>{}, left); break;  // row_bcast:31 into rows 2, 3
    }
  } else {
    switch (s) {
      case 0: Op::move(v, DppMove<0x101, 0xf>{}, left); break;   // row_shl:1
      case 1: Op::move(v, DppMove<0x102, 0xf>{}, left); break;   // row_shl:2
      case 2: Op::move(v, DppMove<0x104, 0xf>{}, left); break;   // row_shl:4
      case 3: Op::move(v, DppMove<0x108, 0xf>{}, left); break;   // row_shl:8
      case 4: Op::move(v, LanePick{row >= 2, 16, 48}, left); break;
      default: Op::move(v, LanePick{row >= 2, 32, 32}, left); break;
    }
  }
  if (s < 4) return in_row >= (1 << s);
  return s == 4 ? (qrow & 1) != 0 : qrow >= 2;
}

// Inclusive scan of the B lane values of a block.  Scan position q = lane
// (FWD) or B-1-lane (reverse).  Inside a wavefront the six Kogge-Stone steps
// of ladder_step move elements between lanes without LDS or barriers; across
// wavefronts (B > 64) only each wavefront's total goes through LDS: lds holds
// B/64 elements, entry-major with row stride B/64.  On exit v is the inclusive
// prefix at q and, when want_ex and has_ex (q > 0), ex the exclusive one.
// Invalid lanes must form a suffix of the scan order: no valid lane reads
// their values.  A wavefront whose lanes are all invalid passes active =
// false (wavefront-uniform): it skips its combines and only takes part in the
// barrier.
template <class Op, int B, bool FWD, typename R>
PKS_DEV void block_ladder(R* lds, typename Op::Elem& v, typename Op::Elem& ex, bool& has_ex, bool active = true,
                          bool want_ex = true) {
  constexpr int NW = B / 64;
  static_assert(B % 64 == 0, "whole wavefronts");
  const int pl = int(threadIdx.x), wl = pl & 63, w = pl >> 6;
  const int qw = FWD ? wl : 63 - wl;        // scan position inside the wavefront
  const int qwave = FWD ? w : NW - 1 - w;   // scan position of the wavefront
  if (active) {
    auto step = [&](int s) {
      typename Op::Elem left;
      if (ladder_step<Op, FWD>(s, wl, v, left)) {
        typename Op::Elem r;
        Op::combine(left, v, r);
        v = r;
      }
    };
    if constexpr (Op::kCompact) {
      // one copy of a long operator instead of six
#pragma unroll 1
      for (int s = 0; s < 6; ++s) step(s);
    } else {
      PKS_UNROLL for (int s = 0; s < 6; ++s) step(s);
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
  if (!active || !want_ex) return;
  // the previous lane's inclusive prefix: wave_shr:1 / wave_shl:1
  if constexpr (FWD) Op::move(v, DppMove<0x138, 0xf>{}, ex);
  else Op::move(v, DppMove<0x130, 0xf>{}, ex);
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
  block_ladder<Op, B, true, R>(lds, v, ex, has_ex, int64_t(lane & ~63) * K < m, K > 1);
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
