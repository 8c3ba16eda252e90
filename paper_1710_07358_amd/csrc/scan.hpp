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
// aggregates in a FIXED tree: tiles form groups of 64, groups of 64 groups,
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

// Wait for a slot of this launch.  The wait is bounded: a correct launch
// never comes close, and once any wait has run out (status set) the others
// stop waiting too, so a broken launch still ends promptly, with the status
// word saying so.
constexpr int kScanSpin = 1 << 16;

template <class Ch, class Item, class IS>
__device__ __forceinline__ Item slot_wait(const uint64_t* slot, uint32_t tag, unsigned* status) {
  constexpr int P = (int)(sizeof(Ch) / 4);
  struct W { uint32_t w[P]; };
  W w;
  uint32_t f = 0;
  for (int spin = 0;; ++spin) {
    bool ok = true;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const uint64_t word = __hip_atomic_load(slot + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ok = ok && (uint32_t)(word >> 33) == tag;
      w.w[i] = (uint32_t)word;
      f = (uint32_t)(word >> 32) & 1u;
    }
    if (ok) break;
    if (spin >= kScanSpin) {
      __hip_atomic_fetch_or(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    if ((spin & 63) == 63 && __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
    __builtin_amdgcn_s_sleep(1);
  }
  return IS::with(__builtin_bit_cast(Ch, w), f);
}

// Slot index of group g at level l (groups of 64^l tiles).
__device__ __forceinline__ int64_t scan_slot(int l, int64_t g) {
  int64_t base = 0, cap = kScanTiles;
  for (int k = 0; k < l; ++k) {
    base += cap;
    cap = (cap + 63) / 64;
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
  unsigned* ctl;          // [0] epoch, [1] next tile, [2] arrivals, [3] status
  int exclusive;
  int aligned;            // x and out are 16-byte aligned
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
  static_assert(OB % 16 == 0, "whole 16-byte stores");

  __shared__ ItA lds_wave[16];
  __shared__ ItC lds_pre;
  __shared__ int64_t lds_tile;
  __shared__ uint32_t lds_heads[SEG ? 1024 * U * V / 32 : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int B = blockDim.x, W = B >> 6;
  const int64_t TE = (int64_t)B * U * V;
  const uint32_t tag = __hip_atomic_load(a.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
  const bool ex = a.exclusive != 0;
  const T* __restrict__ x = (const T*)a.x;
  Out* __restrict__ out = (Out*)a.out;
  const auto combA = [](ItA p, ItA q) { return IA::comb(p, q); };
  const auto combC = [](ItC p, ItC q) { return IC::comb(p, q); };
  const auto to_ch = [](ItA i) { return IC::with((Ch)IA::val(i), IA::flag(i)); };
  const auto to_acc = [](ItC i) { return IA::with((A)IC::val(i), IC::flag(i)); };

  for (;;) {
    if (tid == 0)
      lds_tile = (int64_t)__hip_atomic_fetch_add(a.ctl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t t = lds_tile;
    if (t >= a.ntiles) break;
    const int64_t t0 = t * TE;
    const bool full = a.aligned && (t0 + TE <= a.n);

    // Loads: lane's V elements of each piece (guarded element loads for the
    // last tile or unaligned arrays; past-the-end lanes get the identity).
    u32x4 v[U];
    if (full) {
      const u32x4* p = (const u32x4*)(x + t0) + (int64_t)wave * U * 64 + lane;
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = load16<NT>(p + u * 64);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t base = t0 + ((int64_t)(wave * U + u) * 64 + lane) * V;
        struct E { T e[V]; } e;
#pragma unroll
        for (int k = 0; k < V; ++k) e.e[k] = (base + k < a.n) ? x[base + k] : stored_identity<S, O>();
        v[u] = __builtin_bit_cast(u32x4, e);
      }
    }

    // Segmented: mark the run starts of this tile in an LDS bitmap.
    uint32_t hb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) hb[u] = 0u;
    if constexpr (SEG) {
      for (int i = tid; i < (int)(TE / 32); i += B) lds_heads[i] = 0u;
      __syncthreads();
      const uint64_t fw = a.tile_first[t];
      if ((uint32_t)(fw >> 32) == tag) {
        const int64_t tend = (t0 + TE < a.n) ? t0 + TE : a.n;
        for (int64_t s = (int64_t)(uint32_t)fw + tid; s < a.nheads; s += B) {
          const int64_t p = a.heads[s];
          if (p >= tend) break;
          if (p >= t0) atomicOr(&lds_heads[(p - t0) >> 5], 1u << ((p - t0) & 31));
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int bit = ((wave * U + u) * 64 + lane) * V;
        hb[u] = (lds_heads[bit >> 5] >> (bit & 31)) & ((1u << V) - 1u);
      }
    }

    // Lane totals, then per piece a wavefront scan and the chain of pieces.
    ItA excl[U];
    ItA carry = IA::id();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ItA r = IA::id();
#pragma unroll
      for (int k = 0; k < V; ++k)
        r = IA::comb(IA::make(R::convert(lane_elem<T>(v[u], k)), (hb[u] >> k) & 1u), r);
      const ItA inc = wave_scan_incl(r, IA::id(), combA);
      excl[u] = IA::comb(wave_shift_up(inc, IA::id()), carry);
      carry = IA::comb(readlane(inc, 63), carry);
    }
    if (lane == 0) lds_wave[wave] = carry;
    __syncthreads();
    ItA wp = IA::id();  // prefix of the earlier wavefronts of this tile
    for (int w = 0; w < wave; ++w) wp = IA::comb(lds_wave[w], wp);

    // Wavefront 0: publish the tile's aggregate, fold its exclusive prefix.
    if (wave == 0) {
      ItA agg = IA::id();
      for (int w = 0; w < W; ++w) agg = IA::comb(lds_wave[w], agg);
      const ItC aggc = to_ch(agg);
      if (lane == 0) slot_put<Ch, ItC, IC>(a.slots + kScanSlotWords * scan_slot(0, t), aggc, tag);
      ItC P = IC::id();
      ItC cur = aggc;  // aggregate of this tile's group at the current level
      bool last = true;
      int64_t g = t;
      for (int l = 0; l < kScanLevels; ++l) {
        const int pos = (int)(g & 63);
        const int64_t parent = g >> 6;
        ItC mine = IC::id();
        if (lane < pos)
          mine = slot_wait<Ch, ItC, IC>(a.slots + kScanSlotWords * scan_slot(l, parent * 64 + lane), tag,
                                        a.ctl + 3);
        const ItC F = readlane(wave_scan_incl(mine, IC::id(), combC), 63);
        P = IC::comb(P, F);
        if (last && pos == 63 && l + 1 < kScanLevels) {
          cur = IC::comb(cur, F);
          if (lane == 0) slot_put<Ch, ItC, IC>(a.slots + kScanSlotWords * scan_slot(l + 1, parent), cur, tag);
        } else {
          last = false;
        }
        if (parent == 0) break;
        g = parent;
      }
      if (lane == 0) lds_pre = P;
    }
    __syncthreads();
    const ItC P = lds_pre;

    // Outputs: a left fold from each lane's prefix (the exclusive form
    // reports the value before each element, the neutral element at a run's
    // start).
    struct OE { Out e[V]; };
    OE o[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ItA run = to_acc(IC::comb(to_ch(IA::comb(excl[u], wp)), P));
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const bool h = ((hb[u] >> k) & 1u) != 0;
        const A before = h ? R::identity() : IA::val(run);
        run = IA::comb(IA::make(R::convert(lane_elem<T>(v[u], k)), h), run);
        o[u].e[k] = R::finalize(ex ? before : IA::val(run));
      }
    }
    if (full) {
      struct OV { u32x4 q[OB / 16]; };
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const OV ov = __builtin_bit_cast(OV, o[u]);
        u32x4* dst = (u32x4*)(out + t0) + ((int64_t)(wave * U + u) * 64 + lane) * (OB / 16);
#pragma unroll
        for (int i = 0; i < OB / 16; ++i) {
          if constexpr (NT) __builtin_nontemporal_store(ov.q[i], dst + i);
          else dst[i] = ov.q[i];
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t base = t0 + ((int64_t)(wave * U + u) * 64 + lane) * V;
#pragma unroll
        for (int k = 0; k < V; ++k)
          if (base + k < a.n) out[base + k] = o[u].e[k];
      }
    }
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

template <Store S, Op O, bool SEG> ScanFn scan_pick(bool nt) {
  return nt ? &launch_scan<S, O, SEG, kScanUnroll, true> : &launch_scan<S, O, SEG, kScanUnroll, false>;
}

}  // namespace rd
