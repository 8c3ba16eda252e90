// scan.hpp -- single-pass inclusive / exclusive scan: out[i] is the
// reduction (Section 1.1's combiners) of x over i's run up to i, or strictly
// before i.  A run starts at position 0 and, in the segmented form, at every
// segment offset.  The scan is what the consumers named in the Introduction
// (counting sort, stream compaction, radix sort) build on.
//
// Layout of the work: the array is cut into tiles of block x U x V elements
// (V elements per 16-byte load).  Inside a tile, wavefront w owns U
// consecutive pieces of 64 x V elements; lane l of piece u holds V
// consecutive elements, so each load instruction of the wavefront reads one
// contiguous kilobyte.  A lane folds its V elements, a DPP inclusive scan
// over the 64 lanes gives the exclusive prefix of every lane, the pieces are
// chained in order, and one LDS slot per wavefront and a barrier give each
// wavefront its prefix inside the tile.
//
// Across tiles (single pass: x is read once and out written once) every
// tile publishes its aggregate, and a tile's exclusive prefix is folded from
// aggregates in a FIXED tree: tiles form groups of 8, groups of 8 groups,
// and so on; the last tile of a complete group also publishes the group's
// aggregate.  Tile t's prefix is the fold of its earlier siblings at every
// level.  Because the tree does not depend on timing, float results are the
// same on every run (a classic look-back that stops at whatever prefix is
// ready would not be).  Every wait is for a tile with a smaller index;
// tiles are handed out in increasing order by an atomic counter, so every
// awaited tile belongs to a work-group that is already running.
//
// Published values are tagged with a launch epoch kept in device memory
// (the last work-group advances it), so slots never need clearing and the
// launch can be captured in a graph and replayed.
#pragma once

#include "rd_device.hpp"
#include "rd_internal.hpp"

namespace rd {

// ------------------------------------------------------------------ items

template <class A> struct FlagOf {
  using F = typename std::conditional<sizeof(A) == 8, uint64_t, uint32_t>::type;
};

// Items of the scan.  Plain: the accumulator.  Segmented: (value, head
// flag), where the flag says the span holds the start of a run; combining
// (earlier, later) keeps only the later value when the later span holds a
// start.  That operator is associative, so the same tree serves both.
template <class A, class C, bool SEG> struct ScanItem;

template <class A, class C> struct ScanItem<A, C, false> {
  using I = A;
  static __device__ __forceinline__ I id() { return C::identity(); }
  static __device__ __forceinline__ I make(A v, bool) { return v; }
  static __device__ __forceinline__ I comb(I later, I earlier) { return C::apply(earlier, later); }
  static __device__ __forceinline__ A val(I i) { return i; }
  static __device__ __forceinline__ uint32_t flag(I) { return 0u; }
  static __device__ __forceinline__ I with(A v, uint32_t) { return v; }
};

template <class A, class C> struct ScanItem<A, C, true> {
  using F = typename FlagOf<A>::F;
  struct I {
    A v;
    F f;
  };
  static __device__ __forceinline__ I id() { return I{C::identity(), (F)0}; }
  static __device__ __forceinline__ I make(A v, bool h) { return I{v, (F)(h ? 1 : 0)}; }
  static __device__ __forceinline__ I comb(I later, I earlier) {
    return later.f ? later : I{C::apply(earlier.v, later.v), earlier.f};
  }
  static __device__ __forceinline__ A val(I i) { return i.v; }
  static __device__ __forceinline__ uint32_t flag(I i) { return (uint32_t)i.f; }
  static __device__ __forceinline__ I with(A v, uint32_t f) { return I{v, (F)f}; }
};

// Element type as stored whose conversion is the op's neutral element
// (fills lanes past the end of the array).
template <Store S, Op O> __device__ __forceinline__ typename Stored<S>::T stored_identity() {
  using T = typename Stored<S>::T;
  if constexpr (S == Store::F16) {
    if constexpr (O == Op::Sum) return (T)0x0000u;
    else if constexpr (O == Op::Prod) return (T)0x3C00u;
    else if constexpr (O == Op::Min) return (T)0x7C00u;  // +inf
    else return (T)0xFC00u;                              // -inf
  } else if constexpr (S == Store::BF16) {
    if constexpr (O == Op::Sum) return (T)0x0000u;
    else if constexpr (O == Op::Prod) return (T)0x3F80u;
    else if constexpr (O == Op::Min) return (T)0x7F80u;
    else return (T)0xFF80u;
  } else if constexpr (S == Store::U16) {
    return (T)(O == Op::And ? 0xFFFFu : 0u);
  } else {
    return (T)Combiner<O, T>::identity();
  }
}

// ------------------------------------------------------------------ tagged slots

// A slot holds one published item in two 64-bit words: the high half of
// each word is (epoch tag << 1 | head flag), the low half 32 bits of the
// value.  Words are written and read with agent-scope atomics; a reader
// that sees this launch's tag in every word has the value.
template <class Ch, class Item, class IS>
__device__ __forceinline__ void slot_put(uint64_t* slot, Item it, uint32_t tag) {
  constexpr int P = (int)(sizeof(Ch) / 4);
  struct W { uint32_t w[P]; };
  const W w = __builtin_bit_cast(W, IS::val(it));
  const uint64_t hi = (uint64_t)((tag << 1) | IS::flag(it)) << 32;
#pragma unroll
  for (int i = 0; i < P; ++i)
    __hip_atomic_store(slot + i, hi | (uint64_t)w.w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bound of a wait for published slots: a correct launch never comes
// close.  A wait that runs out sets the sticky status word ctl[3] (read and
// cleared by the host) and writes this launch's tag to ctl[4]; the other
// waits of the same launch see the tag and stop waiting too, so a broken
// launch still ends promptly.  The tag changes with every launch, so a
// later launch is not cut short by an earlier one's give-up.
constexpr int kScanSpin = 1 << 16;

// Wait (in the lanes where `mine` holds) until every word of the slot at
// src carries this launch's tag; w holds the words already loaded.
template <int P>
__device__ __forceinline__ void scan_wait(uint64_t (&w)[P], const uint64_t* src, bool mine, uint32_t tag,
                                          unsigned* ctl) {
  for (int spin = 0;; ++spin) {
    bool ok = true;
#pragma unroll
    for (int i = 0; i < P; ++i) ok = ok && (!mine || (uint32_t)(w[i] >> 33) == tag);
    if (ok) break;
    if (spin >= kScanSpin) {
      __hip_atomic_fetch_or(ctl + 3, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ctl + 4, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    if ((spin & 63) == 63 && __hip_atomic_load(ctl + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag) break;
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (mine && (uint32_t)(w[i] >> 33) != tag)
        w[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Slot index of the aggregate of group g at level l (groups of kScanFan^l
// tiles).
__device__ __forceinline__ int64_t scan_slot(int l, int64_t g) {
  int64_t base = 0, cap = kScanTiles;
  for (int k = 0; k < l; ++k) {
    base += cap;
    cap = (cap + kScanFan - 1) / kScanFan;
  }
  return base + g;
}

// ------------------------------------------------------------------ kernels

struct ScanArgs {
  const void* x;
  void* out;
  int64_t n;
  const int64_t* heads;   // segmented: run starts (nondecreasing), else null
  int64_t nheads;
  int64_t ntiles;
  uint64_t* slots;        // kScanSlots slots of kScanSlotWords words
  uint64_t* tile_first;   // segmented: per tile, tagged index of its first head
  unsigned* ctl;          // [0] epoch, [1] next tile, [2] arrivals, [3] status, [4] give-up tag
  int exclusive;
  int aligned;            // x and out are 16-byte aligned
  int probe;              // failure-path test: one wait for the never-published slot of tile ntiles
};

// Per tile of the segmented form: the index of the first head that falls in
// it, tagged with the epoch of the scan launch that follows.  (A template
// only so that every translation unit may instantiate it.)
template <int = 0>
__global__ __launch_bounds__(256) void scan_heads_kernel(const int64_t* __restrict__ heads, int64_t nheads,
                                                         int64_t n, int64_t tile_elems,
                                                         uint64_t* __restrict__ tile_first,
                                                         unsigned* __restrict__ ctl) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nheads) return;
  const int64_t p = heads[s];
  if (p < 0 || p >= n) return;
  const int64_t t = p / tile_elems;
  if (s > 0) {
    const int64_t q = heads[s - 1];
    if (q >= t * tile_elems && q <= p) return;  // an earlier head of the same tile
  }
  const unsigned e = __hip_atomic_load(ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  tile_first[t] = ((uint64_t)(e + 1u) << 32) | (uint64_t)(uint32_t)s;
}

// One lane's V elements of each of its U pieces of tile t0 .. t0 + TE:
// 16-byte loads when the tile is whole and aligned, else guarded element
// loads with the neutral element past the end.
template <Store S, Op O, int U, bool NT>
__device__ __forceinline__ void tile_load(const typename Stored<S>::T* __restrict__ x, int64_t n, int64_t t0,
                                          int64_t TE, bool aligned, int wave, int lane, u32x4 (&v)[U]) {
  using T = typename Stored<S>::T;
  constexpr int V = 16 / (int)sizeof(T);
  if (aligned && t0 + TE <= n) {
    const u32x4* p = (const u32x4*)(x + t0) + (int64_t)wave * U * 64 + lane;
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load16<NT>(p + u * 64);
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t base = t0 + ((int64_t)(wave * U + u) * 64 + lane) * V;
      struct E { T e[V]; } e;
#pragma unroll
      for (int k = 0; k < V; ++k) e.e[k] = (base + k < n) ? x[base + k] : stored_identity<S, O>();
      v[u] = __builtin_bit_cast(u32x4, e);
    }
  }
}

// Segmented form: set the bit of every run start of tile t in `bits`
// (cleared beforehand).  Starts come from the tagged first-head index of
// the tile and the offsets that follow it.
__device__ __forceinline__ void mark_heads(const ScanArgs& a, int64_t t, int64_t t0, int64_t TE, uint32_t tag,
                                           uint32_t* bits) {
  const uint64_t fw = a.tile_first[t];
  if ((uint32_t)(fw >> 32) != tag) return;
  const int64_t tend = (t0 + TE < a.n) ? t0 + TE : a.n;
  for (int64_t s = (int64_t)(uint32_t)fw + threadIdx.x; s < a.nheads; s += blockDim.x) {
    const int64_t p = a.heads[s];
    if (p >= tend) break;
    if (p >= t0) atomicOr(&bits[(p - t0) >> 5], 1u << ((p - t0) & 31));
  }
}

__device__ __forceinline__ unsigned grab_tile(unsigned* ctl) {
  return __hip_atomic_fetch_add(ctl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <Store S, Op O, bool SEG, int U, bool NT>
__global__ __launch_bounds__(1024) void scan_kernel(ScanArgs a) {
  using R = Red<S, O>;
  using T = typename R::T;
  using A = typename R::Acc;
  using Out = typename R::Out;
  // Values that cross tiles: float sums travel in float64 (the chain of
  // tile prefixes then adds no float32 rounding), everything else as is.
  using Ch = typename std::conditional<std::is_same<A, float>::value && O == Op::Sum, double, A>::type;
  using IA = ScanItem<A, Combiner<O, A>, SEG>;
  using IC = ScanItem<Ch, Combiner<O, Ch>, SEG>;
  using ItA = typename IA::I;
  using ItC = typename IC::I;
  constexpr int V = 16 / (int)sizeof(T);
  constexpr int OB = V * (int)sizeof(Out);  // output bytes per lane and piece: 16 or 32
  constexpr int P = (int)(sizeof(Ch) / 4);  // words per published slot
  constexpr int HW = SEG ? 1024 * U * V / 32 : 1;
  static_assert(OB % 16 == 0, "whole 16-byte stores");

  __shared__ ItA lds_wave[16];
  __shared__ ItC lds_pre;
  __shared__ int64_t lds_next[2];
  __shared__ uint32_t lds_heads[SEG ? 2 : 1][HW];

  // The wavefront index is the same in every lane; saying so keeps the
  // tile bookkeeping in scalar registers.
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int B = blockDim.x, W = B >> 6;
  const int64_t TE = (int64_t)B * U * V;
  const uint32_t tag = __hip_atomic_load(a.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
  const bool ex = a.exclusive != 0;
  const bool aligned = a.aligned != 0;
  const T* __restrict__ x = (const T*)a.x;
  Out* __restrict__ out = (Out*)a.out;
  // Head bits of a lane: V bits per piece, piece u at bit u * V.
  using HB = typename std::conditional<(U * V > 32), uint64_t, uint32_t>::type;
  using IP = ScanItem<A, Combiner<O, A>, false>;  // items of a piece without run starts
  const auto combA = [](ItA p, ItA q) { return IA::comb(p, q); };
  const auto combP = [](A p, A q) { return IP::comb(p, q); };
  const auto combC = [](ItC p, ItC q) { return IC::comb(p, q); };
  const auto to_ch = [](ItA i) { return IC::with((Ch)IA::val(i), IA::flag(i)); };
  const auto to_acc = [](ItC i) { return IA::with((A)IC::val(i), IC::flag(i)); };
  const auto piece_bits = [](HB hb, int u) -> uint32_t {
    return SEG ? (uint32_t)(hb >> (u * V)) & ((1u << V) - 1u) : 0u;
  };

  // Lane totals of one tile, a wavefront scan per piece and the chain of
  // pieces: excl[u] is the lane's exclusive prefix inside its wavefront's
  // part of the tile, the return value the wavefront's aggregate.  A piece
  // in which no lane holds a run start (bit u of `quiet`, the same in every
  // lane) is scanned on bare values: with every flag clear the (value, flag)
  // combine performs the same operations in the same order, so the result
  // is identical, and runs are typically far longer than a piece.
  const auto tile_scan = [&](const u32x4 (&v)[U], HB hb, ItA (&excl)[U], uint32_t& quiet) {
    ItA carry = IA::id();
    quiet = 0u;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t pb = piece_bits(hb, u);
      if (!SEG || __builtin_amdgcn_ballot_w64(pb != 0u) == 0ull) {
        A r = IP::id();
#pragma unroll
        for (int k = 0; k < V; ++k) r = IP::comb(R::convert(lane_elem<T>(v[u], k)), r);
        const A inc = wave_scan_incl(r, IP::id(), combP);
        excl[u] = IA::comb(IA::with(wave_shift_up(inc, IP::id()), 0u), carry);
        carry = IA::comb(IA::with(readlane(inc, 63), 0u), carry);
        quiet |= 1u << u;
      } else {
        ItA r = IA::id();
#pragma unroll
        for (int k = 0; k < V; ++k) r = IA::comb(IA::make(R::convert(lane_elem<T>(v[u], k)), (pb >> k) & 1u), r);
        const ItA inc = wave_scan_incl(r, IA::id(), combA);
        excl[u] = IA::comb(wave_shift_up(inc, IA::id()), carry);
        carry = IA::comb(readlane(inc, 63), carry);
      }
    }
    return carry;
  };
  const auto head_bits = [&](const uint32_t* bits) -> HB {
    HB hb = 0;
    if constexpr (SEG) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int bit = ((wave * U + u) * 64 + lane) * V;
        hb |= (HB)((bits[bit >> 5] >> (bit & 31)) & ((1u << V) - 1u)) << (u * V);
      }
    }
    return hb;
  };

  // Wavefront 0's look-back state for the current tile.  Lane
  // kScanFan * l + j reads the aggregate of sibling j at level l of the tree
  // (all levels in one load, issued as soon as the tile's own aggregate is
  // out); the waits come later, level by level.
  const int my_l = lane >> kScanFanLog, my_j = lane & (kScanFan - 1);
  uint64_t lw[P];
  bool lact = false;
  const uint64_t* lsrc = a.slots;
  ItC aggc = IC::id();
  const auto publish_and_ask = [&](int64_t tt) {
    ItA agg = IA::id();
    for (int w = 0; w < W; ++w) agg = IA::comb(lds_wave[w], agg);
    aggc = to_ch(agg);
    if (lane == 0) slot_put<Ch, ItC, IC>(a.slots + kScanSlotWords * scan_slot(0, tt), aggc, tag);
    const int64_t my_g = my_l < kScanLevels ? (tt >> (kScanFanLog * my_l)) : 0;
    lact = my_l < kScanLevels && (my_l == 0 || my_g != 0) && my_j < (int)(my_g & (kScanFan - 1));
    lsrc = a.slots + kScanSlotWords * scan_slot(my_l < kScanLevels ? my_l : 0, (my_g >> kScanFanLog) * kScanFan + my_j);
#pragma unroll
    for (int i = 0; i < P; ++i)
      lw[i] = lact ? __hip_atomic_load(lsrc + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
  };
  // Fold the tile's exclusive prefix; a tile that completes a group
  // publishes the group's aggregate as soon as that level is in, so group
  // aggregates never wait for anything above them.
  const auto finish_lookback = [&](int64_t tt) {
    ItC Pre = IC::id();
    ItC cur = aggc;
    bool last = true;
    int64_t g = tt;
    for (int l = 0; l < kScanLevels; ++l) {
      if (l > 0 && g == 0) break;  // no earlier groups at this level or above
      scan_wait<P>(lw, lsrc, lact && my_l == l, tag, a.ctl);
      struct Wd { uint32_t q[P]; } wd;
#pragma unroll
      for (int i = 0; i < P; ++i) wd.q[i] = (uint32_t)lw[i];
      const ItC got = (lact && my_l == l) ? IC::with(__builtin_bit_cast(Ch, wd), (uint32_t)(lw[0] >> 32) & 1u)
                                          : IC::id();
      const ItC F = readlane(wave_scan_incl(got, IC::id(), combC), 63);
      Pre = IC::comb(Pre, F);
      last = last && (g & (kScanFan - 1)) == kScanFan - 1;
      if (last && l + 1 < kScanLevels) {
        cur = IC::comb(cur, F);
        if (lane == 0)
          slot_put<Ch, ItC, IC>(a.slots + kScanSlotWords * scan_slot(l + 1, g >> kScanFanLog), cur, tag);
      }
      g >>= kScanFanLog;
    }
    return Pre;
  };

  // Pipeline.  Rule: between taking a tile and publishing its aggregate a
  // work-group never waits for another tile (otherwise the aggregates of
  // later tiles would wait on earlier look-backs: a chain along the array).
  // So a tile is taken only after the previous tile's prefix is known, and
  // its loads overlap the previous tile's stores.
  if (a.probe && blockIdx.x == 0 && wave == 0) {
    // Failure-path test: wait for the aggregate of tile ntiles, which no tile
    // of this launch publishes (the host ensures ntiles < kScanTiles), so the
    // wait runs out and the launch reports it.
    const uint64_t* src = a.slots + kScanSlotWords * scan_slot(0, a.ntiles);
    uint64_t pw[P];
#pragma unroll
    for (int i = 0; i < P; ++i) pw[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    scan_wait<P>(pw, src, lane == 0, tag, a.ctl);
  }
  if (tid == 0) lds_next[0] = grab_tile(a.ctl);
  if constexpr (SEG)
    for (int i = tid; i < (int)(TE / 32); i += B) lds_heads[0][i] = 0u;
  __syncthreads();
  int64_t t = lds_next[0];
  u32x4 v[U];
  HB hb = 0;
  uint32_t quiet = 0u;
  ItA excl[U];
  ItA wp = IA::id();
  if (t < a.ntiles) {
    tile_load<S, O, U, NT>(x, a.n, t * TE, TE, aligned, wave, lane, v);
    if constexpr (SEG) {
      mark_heads(a, t, t * TE, TE, tag, lds_heads[0]);
      __syncthreads();
    }
    hb = head_bits(lds_heads[0]);
    const ItA wagg = tile_scan(v, hb, excl, quiet);
    if (lane == 0) lds_wave[wave] = wagg;
    __syncthreads();
    for (int w = 0; w < wave; ++w) wp = IA::comb(lds_wave[w], wp);
    if (wave == 0) publish_and_ask(t);
  }
  int it = 0;
  while (t < a.ntiles) {
    const int nx = (it + 1) & 1;
    const int64_t t0 = t * TE;
    if (wave == 0) {
      const ItC Pre = finish_lookback(t);
      if (lane == 0) {
        lds_pre = Pre;
        lds_next[nx] = grab_tile(a.ctl);
      }
    }
    if constexpr (SEG)
      for (int i = tid; i < (int)(TE / 32); i += B) lds_heads[nx][i] = 0u;
    __syncthreads();
    const ItC Pt = lds_pre;
    const int64_t tn = lds_next[nx];
    u32x4 vn[U];
    if (tn < a.ntiles) {
      tile_load<S, O, U, NT>(x, a.n, tn * TE, TE, aligned, wave, lane, vn);
      if constexpr (SEG) mark_heads(a, tn, tn * TE, TE, tag, lds_heads[nx]);
    }

    // Outputs of t: a left fold from each lane's prefix (the exclusive form
    // reports the value before each element, the neutral element at a run's
    // start).
    struct OE { Out e[V]; };
    const bool whole = aligned && t0 + TE <= a.n;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ItA run = to_acc(IC::comb(to_ch(IA::comb(excl[u], wp)), Pt));
      OE o;
      if (!SEG || ((quiet >> u) & 1u) != 0u) {
        A rv = IA::val(run);
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const A before = rv;
          rv = IP::comb(R::convert(lane_elem<T>(v[u], k)), rv);
          o.e[k] = R::finalize(ex ? before : rv);
        }
      } else {
        const uint32_t pb = piece_bits(hb, u);
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const bool h = ((pb >> k) & 1u) != 0;
          const A before = h ? R::identity() : IA::val(run);
          run = IA::comb(IA::make(R::convert(lane_elem<T>(v[u], k)), h), run);
          o.e[k] = R::finalize(ex ? before : IA::val(run));
        }
      }
      const int64_t base = t0 + ((int64_t)(wave * U + u) * 64 + lane) * V;
      if (whole) {
        struct OV { u32x4 q[OB / 16]; };
        const OV ov = __builtin_bit_cast(OV, o);
        u32x4* dst = (u32x4*)(out + base);
#pragma unroll
        for (int i = 0; i < OB / 16; ++i) {
          if constexpr (NT) __builtin_nontemporal_store(ov.q[i], dst + i);
          else dst[i] = ov.q[i];
        }
      } else {
#pragma unroll
        for (int k = 0; k < V; ++k)
          if (base + k < a.n) out[base + k] = o.e[k];
      }
    }

    // The next tile: its scan and aggregate, published at once.
    if constexpr (SEG) __syncthreads();  // its run starts are marked
    if (tn < a.ntiles) {
      hb = head_bits(lds_heads[SEG ? nx : 0]);
      const ItA wagg = tile_scan(vn, hb, excl, quiet);
      if (lane == 0) lds_wave[wave] = wagg;
    }
    __syncthreads();
    if (tn < a.ntiles) {
      wp = IA::id();
      for (int w = 0; w < wave; ++w) wp = IA::comb(lds_wave[w], wp);
      if (wave == 0) publish_and_ask(tn);
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = vn[u];
    }
    t = tn;
    ++it;
  }

  // The last work-group out re-arms the counters and advances the epoch.
  if (tid == 0) {
    const unsigned prev = __hip_atomic_fetch_add(a.ctl + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x - 1) {
      const unsigned e = __hip_atomic_load(a.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(a.ctl + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(a.ctl + 2, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(a.ctl + 0, e + 1u >= kScanEpochs ? 0u : e + 1u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <Store S, Op O, bool SEG, int U, bool NT>
hipError_t launch_scan(const ScanCall& c, const Scratch& ws, const Launch& l, hipStream_t s) {
  using T = typename Stored<S>::T;
  constexpr int V = 16 / (int)sizeof(T);
  const int64_t te = (int64_t)l.block * U * V;
  ScanArgs a;
  a.x = c.x;
  a.out = c.out;
  a.n = c.n;
  a.heads = c.heads;
  a.nheads = SEG ? c.nheads : 0;
  a.ntiles = (c.n + te - 1) / te;
  a.slots = ws.scan_slots;
  a.tile_first = ws.scan_tile_first;
  a.ctl = ws.scan_ctl;
  a.exclusive = c.exclusive ? 1 : 0;
  a.aligned = (((uintptr_t)c.x | (uintptr_t)c.out) & 15u) == 0 ? 1 : 0;
  a.probe = (l.probe && a.ntiles < kScanTiles) ? 1 : 0;
  if (SEG && a.nheads > 0) {
    const int64_t blocks = (a.nheads + 255) / 256;
    hipLaunchKernelGGL(scan_heads_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, s, c.heads, a.nheads, c.n, te,
                       ws.scan_tile_first, ws.scan_ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int grid = (int)(a.ntiles < l.grid ? a.ntiles : l.grid);
  hipLaunchKernelGGL((scan_kernel<S, O, SEG, U, NT>), dim3(grid), dim3(l.block), 0, s, a);
  return hipGetLastError();
}

template <Store S, Op O, bool SEG> ScanFn scan_pick(int u, bool nt) {
  if (u == 4) return nt ? &launch_scan<S, O, SEG, 4, true> : &launch_scan<S, O, SEG, 4, false>;
  if (u == 8) return nt ? &launch_scan<S, O, SEG, 8, true> : &launch_scan<S, O, SEG, 8, false>;
  return nullptr;
}

}  // namespace rd
