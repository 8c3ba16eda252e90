// reduce_segmented.hpp -- many segments, one persistent launch (gfx950).
//
// out[s] = x[offsets[s]] (+) ... (+) x[offsets[s+1]-1].
//
// Persistent threads suit irregular work (Section 2.5), so the launch holds a
// fixed grid and the work is split by elements, not by segments.  The
// range [offsets[0], offsets[nseg]) is cut into windows of 64 x U sixteen-byte
// vectors; each work-group owns a contiguous run of windows and deals them
// to its wavefronts round-robin (round r: wavefront j takes window r*WB + j),
// so the wavefronts of a work-group read adjacent memory at the same time --
// the access order of the plain kernel.  (Giving each wavefront one long
// contiguous run instead costs 10-15% of read bandwidth on this GPU.)
//
// A wavefront folds its window while tracking the segment it is in
// (wavefront-uniform state plus a register cache of 64 offsets); a window
// inside one segment is folded straight into the private accumulators, a
// window that crosses segment ends is folded one segment at a time with
// per-element selects (never a multiply-by-flag, Section 3).  A segment
// wholly inside a window is written at once.  The window's first piece (of a
// segment that began earlier) and last piece (of one that runs on) go to an
// LDS entry; every 256 windows wavefront 0 joins the entries in window order
// with a segmented wavefront scan, writing each segment that ends there.  A
// segment that reaches the wavefront's next window is not reduced at the
// window's end: its elements stay in the accumulators across windows, so a
// long segment costs one wavefront reduction per wavefront, not per window.
// A segment that crosses work-groups leaves one partial per work-group; each
// work-group bumps a counter owned by the segment's first work-group, and the
// one that completes the count folds the partials in work-group order and
// writes the result.  Every fold order is fixed by the launch shape, so the
// result is deterministic.  Empty segments are written with the neutral
// element by a grid-stride pass at the end.
#pragma once

#include "rd_device.hpp"
#include "rd_internal.hpp"

namespace rd {

namespace {

__device__ __forceinline__ int64_t rl64(int64_t v, int lane) { return readlane(v, lane); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// A running piece in the join of window entries: value and restart flag.
// Combining (earlier, later) keeps only the later value when the later
// entry restarts (a segment ended in it); the operator is associative.
template <class A> struct SegRun {
  using F = typename std::conditional<sizeof(A) == 8, uint64_t, uint32_t>::type;
  A v;
  F f;
};

}  // namespace

// Windows of the range [lo, hi): the aligned vectors [A, A + nvec*V) in
// windows of 64*U vectors (the last one may be short); the unaligned head
// [lo, A) joins window 0 and the ragged tail joins the last window.
struct SegWindows {
  int64_t lo, hi, A, nvec, win, nw, per_block;
  int V;
  __device__ int64_t begin(int64_t wi) const { return wi == 0 ? lo : A + wi * win * V; }
  __device__ int64_t end(int64_t wi) const {
    return wi == nw - 1 ? hi : A + min((wi + 1) * win, nvec) * V;
  }
  __device__ int64_t window_of(int64_t pos) const {
    if (pos < A) return 0;
    return min((pos - A) / V / win, nw - 1);
  }
  __device__ int64_t block_of(int64_t pos) const { return window_of(pos) / per_block; }
};

template <class R, int U, bool NT>
__global__ __launch_bounds__(1024) void segmented_kernel(const typename R::T* __restrict__ x,
                                                         const int64_t* __restrict__ offsets,
                                                         int64_t nseg,
                                                         typename R::Out* __restrict__ out,
                                                         uint64_t* __restrict__ carry,
                                                         unsigned* __restrict__ counters,
                                                         unsigned* __restrict__ status) {
  using T = typename R::T;
  using A = typename R::Acc;
  using Run = SegRun<A>;
  constexpr int V = 16 / (int)sizeof(T);
  constexpr int K = U * V;  // elements per lane per window
  const int lane = threadIdx.x & 63;
  // The wavefront index is the same in every lane; saying so keeps all
  // window and segment bookkeeping in scalar registers.
  const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), WB = blockDim.x >> 6;
  constexpr int NE = 256;  // LDS entries (windows) per batch
  const int D = NE / WB;   // rounds per batch

  // Empty segments get the neutral element (no other path writes them:
  // the walk over segments skips them).  Done last, so its loads do not
  // delay the first data loads.
  const auto fill_empty = [&]() {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nseg; s += stride)
      if (offsets[s + 1] <= offsets[s]) out[s] = R::finalize(R::identity());
  };

  SegWindows P;
  P.lo = offsets[0];
  P.hi = offsets[nseg];
  if (P.hi <= P.lo) {
    fill_empty();
    return;
  }
  P.V = V;
  {
    const uintptr_t a = (uintptr_t)(x + P.lo);
    const int64_t head = (int64_t)(((16u - (unsigned)(a & 15u)) & 15u) / sizeof(T));
    P.A = min(P.lo + head, P.hi);
    P.nvec = (P.hi - P.A) / V;
    P.win = 64 * U;
    P.nw = P.nvec > 0 ? (P.nvec + P.win - 1) / P.win : 1;
    P.per_block = (P.nw + gridDim.x - 1) / gridDim.x;
  }
  const int64_t wfirst = (int64_t)blockIdx.x * P.per_block;
  const int64_t wlast = min(wfirst + P.per_block, P.nw);  // this work-group's windows: [wfirst, wlast)
  const int64_t rounds = (P.per_block + WB - 1) / WB;
  const int64_t batches = (rounds + D - 1) / D;

  // LDS entries of two batches: per window, the piece of the segment that
  // began before it (head; `cover` if that segment also runs past it) and
  // the piece of the segment that runs past it (tail).
  __shared__ int64_t e_hsid[2][NE], e_tsid[2][NE];
  __shared__ A e_hval[2][NE], e_tval[2][NE];
  __shared__ int e_flags[2][NE];  // bit 0 head, bit 1 cover, bit 2 tail

  const u32x4* xv = (const u32x4*)(x + P.A);
  auto load_window = [&](int64_t wi, u32x4 (&raw)[U]) {
    const int64_t vb = wi * P.win;
    const int64_t nv = min(P.win, P.nvec - vb);
    if (nv == P.win) {
#pragma unroll
      for (int u = 0; u < U; ++u) raw[u] = load16<NT>(xv + vb + u * 64 + lane);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        raw[u] = u32x4{0u, 0u, 0u, 0u};
        if (u * 64 + lane < nv) raw[u] = load16<NT>(xv + vb + u * 64 + lane);
      }
    }
  };

  // ---- segment tracking (wavefront-uniform): s is the segment at the
  // current position, [seg_begin, seg_end) its extent.
  int64_t s = 0, seg_begin = 0, seg_end = 0;
  // Largest i in [a, nseg-1] with offsets[i] <= pos (offsets[a] <= pos holds): 64-ary search.
  auto search = [&](int64_t a, int64_t pos) -> int64_t {
    int64_t b = nseg - 1;
    while (b - a >= 64) {
      const int64_t step = (b - a + 63) / 64;
      const int64_t idx = min(a + (int64_t)lane * step, b);
      const uint64_t m = ballot(offsets[idx] <= pos);  // prefix of lanes (offsets sorted)
      const int k = __builtin_popcountll(m) - 1;       // >= 0 since lane 0 holds offsets[a]
      const int64_t na = min(a + (int64_t)k * step, b);  // probes past b were clamped to b
      b = min(na + step - 1, b);
      a = na;
    }
    const int64_t idx = min(a + (int64_t)lane, b);
    const uint64_t m = ballot(a + lane <= b && offsets[idx] <= pos);
    return a + __builtin_popcountll(m) - 1;
  };
  // Register cache of offsets[cbase .. cbase+63] (indices clamped to nseg).
  int64_t cbase = -128, cache = 0;  // empty until the first offset_at
  auto offset_at = [&](int64_t j) -> int64_t {  // j in [0, nseg]; wavefront-uniform
    if (j < cbase || j >= cbase + 64) {
      cbase = j;
      cache = offsets[min(cbase + lane, nseg)];
    }
    return rl64(cache, (int)(j - cbase));
  };
  // Move s forward to the segment holding pos (pos >= seg_begin).
  auto seek = [&](int64_t pos) {
    int64_t i = s;
    for (int hop = 0; i < nseg - 1; ++hop) {
      if (offset_at(i + 1) > pos) break;  // still inside (the common case)
      if (hop == 2) {                      // far ahead: search instead of walking the cache
        i = search(i + 1, pos);
        break;
      }
      const int64_t j = cbase + lane;
      const uint64_t m = ballot(j >= i + 1 && j <= nseg - 1 && cache <= pos);
      i += __builtin_popcountll(m);
      if (!(m >> 63)) break;  // the run of offsets <= pos ended inside the cache
    }
    if (i != s) {
      s = i;
      seg_begin = offset_at(s);
    }
    seg_end = offset_at(s + 1);
  };
  // Next nonempty segment after s: the largest i with offsets[i] <= pos (= end of s).
  auto next_segment = [&](int64_t cur, int64_t pos) -> int64_t {
    int64_t i = cur + 1;  // offsets[cur+1] == pos
    while (i < nseg - 1) {
      (void)offset_at(i + 1);
      const int64_t j = cbase + lane;
      const uint64_t m = ballot(j >= i + 1 && j <= nseg - 1 && cache <= pos);
      const int cnt = __builtin_popcountll(m);
      i += cnt;
      if (cnt == 0 || !(m >> 63)) break;  // run ended inside the cache
    }
    return i;
  };

  A acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = R::identity();
  auto fold_acc = [&]() -> A {
    A v = acc[0];
#pragma unroll
    for (int k = 1; k < K; ++k) v = R::apply(v, acc[k]);
    return wave_reduce_r<R>(v);
  };

  // The current window [r0, r1) and its two pieces.
  int64_t r0 = 0, r1 = 0;
  int64_t head_sid = -1, tail_sid = -1;
  A head_val = R::identity(), tail_val = R::identity();
  bool head_cover = false;
  // Piece of segment `sid` covering [sb, se) from this window's view:
  // written at once when the segment lies inside the window.
  auto emit = [&](int64_t sid, A piece, int64_t sb, int64_t se) {
    if (sb >= r0 && se <= r1) {
      if (lane == 0) out[sid] = R::finalize(piece);
    } else if (sb < r0) {
      head_sid = sid;
      head_val = piece;
      head_cover = se > r1;
    } else {
      tail_sid = sid;
      tail_val = piece;
    }
  };

  // Fold elements vals[k] at window-relative positions rel(k) into the
  // segments they belong to.  Span = [P0, wend).
  auto consume = [&](const A (&vals)[K], auto rel, int64_t P0, int64_t wend) {
    int64_t consumed = P0;
    bool carried = true;  // acc[] holds segment s's piece from earlier windows until s ends here
    while (seg_end < wend) {
      // This lane's part of segment s: the carried piece (at s's end only),
      // then the elements at window-relative positions [from, from + len),
      // tested with one unsigned compare each.
      const uint32_t from = (uint32_t)(consumed - P0), len = (uint32_t)(seg_end - consumed);
      A lane_v = R::identity();
      if (carried) {
        lane_v = acc[0];
#pragma unroll
        for (int k = 1; k < K; ++k) lane_v = R::apply(lane_v, acc[k]);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = R::identity();
        carried = false;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t q = (uint32_t)rel(k) - from;
        lane_v = R::apply(lane_v, q < len ? vals[k] : R::identity());
      }
      emit(s, wave_reduce_r<R>(lane_v), seg_begin, seg_end);
      consumed = seg_end;
      s = next_segment(s, seg_end);
      seg_begin = consumed;
      seg_end = offset_at(s + 1);
    }
    // The piece of the segment that runs on joins the accumulators.
    const int32_t from = (int32_t)(consumed - P0);
    if (from == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = R::apply(acc[k], vals[k]);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const A v = rel(k) >= from ? vals[k] : R::identity();
        acc[k] = R::apply(acc[k], v);
      }
    }
  };

  // Scalar span (unaligned head or ragged tail): one element per lane, positions P0 + lane.
  auto consume_scalar = [&](int64_t P0, int64_t wend) {
    A vals[K];
#pragma unroll
    for (int k = 0; k < K; ++k) vals[k] = R::identity();
    if (P0 + lane < wend) vals[0] = R::convert(x[P0 + lane]);
    consume(vals, [&](int k) { return k == 0 ? (int32_t)lane : (int32_t)0x7FFFFFFF; }, P0, wend);
  };
  auto rel_vec = [&](int k) { return (int32_t)(((k / V) * 64 + lane) * V + (k % V)); };

  // ---- wavefront 0's join of the entries, carried across batches: the
  // running piece (value, segment, whether that segment began before this
  // work-group) after the last joined window.
  Run jrun{R::identity(), 0};
  int64_t jsid = -1;
  bool jbefore = true;
  auto block_emit = [&](int64_t sid, A piece, bool before, bool ends_here) {
    constexpr int SW = slot_words<A>();
    static_assert(SW <= kCarryWords, "carry slot too small");
    const int64_t blk = blockIdx.x;
    if (!before && ends_here) {
      if (lane == 0) out[sid] = R::finalize(piece);
      return;
    }
    const int64_t bf = P.block_of(offsets[sid]), bl = P.block_of(offsets[sid + 1] - 1);
    const unsigned np = (unsigned)(bl - bf + 1);
    const int64_t slot = before ? 2 * blk : 2 * blk + 1;
    unsigned prev = 0;
    if (lane == 0) {
      publish(carry + slot * SW, piece);
      prev = __hip_atomic_fetch_add(counters + bf, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = (unsigned)__builtin_amdgcn_readfirstlane((int)prev);
    if (prev + 1 != np) return;
    // Last piece counted in: fold bf's tail slot and the head slots of
    // bf+1..bl, in that order, each lane waiting for its slot's tag.
    A total = R::identity();
    for (int64_t base = 0; base < (int64_t)np; base += 64) {
      const int64_t q = base + lane;
      A v = R::identity();
      if (q < (int64_t)np) {
        const int64_t bb = bf + q;
        v = collect<A>(carry + (q == 0 ? 2 * bb + 1 : 2 * bb) * SW, status);
      }
      total = R::apply(total, wave_reduce_r<R>(v));
    }
    if (lane == 0) {
      out[sid] = R::finalize(total);
      __hip_atomic_store(counters + bf, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  // Join 64 entries of a batch, from entry c: lane e holds window c + e, in order.
  auto join = [&](int b, int c) {
    const auto comb = [](Run later, Run earlier) {
      return later.f ? later : Run{R::apply(earlier.v, later.v), earlier.f};
    };
    const int fl = e_flags[b][c + lane];
    const bool hh = (fl & 1) != 0, cov = (fl & 2) != 0, ht = (fl & 4) != 0;
    const A hv = e_hval[b][c + lane];
    const int64_t hs = e_hsid[b][c + lane];
    // A window that is not covered ends the running piece (after adding its
    // head) and starts its tail, if any.
    const bool rs = !cov;
    const Run item{rs ? (ht ? e_tval[b][c + lane] : R::identity()) : (hh ? hv : R::identity()),
                   (typename Run::F)(rs ? 1 : 0)};
    const Run inc = wave_scan_incl(item, Run{R::identity(), 0}, comb);
    const Run prev = comb(wave_shift_up(inc, Run{R::identity(), 0}), jrun);  // running piece before window e
    const uint64_t restarts = ballot(rs);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const bool before = jbefore && (restarts & below) == 0ull;
    const bool ends = hh && !cov;
    const A total = R::apply(prev.v, hv);
    if (ends && !before) out[hs] = R::finalize(total);
    const uint64_t gm = ballot(ends && before);  // the segment that began before this work-group
    if (gm != 0ull) {
      const int l = __builtin_ctzll(gm);
      block_emit(rl64(hs, l), readlane(total, l), true, true);
    }
    jrun = comb(readlane(inc, 63), jrun);
    if (restarts != 0ull) {
      const int l = 63 - __builtin_clzll(restarts);
      jsid = ((ballot(ht) >> l) & 1ull) != 0ull ? rl64(e_tsid[b][c + lane], l) : -1;
      jbefore = false;
    } else if (jsid < 0) {
      const uint64_t hm = ballot(hh);
      if (hm != 0ull) jsid = rl64(hs, __builtin_ctzll(hm));
    }
  };

  // ---- the rounds
  int64_t wi = wfirst + wib;  // this wavefront's first window
  u32x4 cur[U], nxt[U];
  if (wi < wlast) {
    if (wi * P.win < P.nvec) load_window(wi, cur);
    s = search(0, P.begin(wi));
    seg_begin = offsets[s];
    seg_end = offset_at(s + 1);
  }
  for (int64_t bt = 0; bt < batches; ++bt) {
    const int b = (int)(bt & 1);
    for (int rr = 0; rr < D; ++rr, wi += WB) {
      int flags = 2;  // no window: passes the running piece on
      if (wi < wlast) {
        const int64_t wn = wi + WB;
        if (wn < wlast && wn * P.win < P.nvec) load_window(wn, nxt);
        const int64_t vb = wi * P.win;
        r0 = P.A + vb * V;  // an inner window: full, no unaligned head or ragged tail
        r1 = r0 + P.win * V;
        const bool inner = wi != 0 && wi != P.nw - 1;
        if (inner && seg_end <= r0) seek(r0);  // a segment ended in another wavefront's window
        if (inner && seg_begin < r0 && seg_end >= r1) {
          // The common case: the whole window lies in segment s, which began
          // before it -- fold it and decide whether s must be reported here.
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e)
              acc[u * V + e] = R::apply(acc[u * V + e], R::convert(lane_elem<T>(cur[u], e)));
          if (wn < wlast && seg_end > P.A + wn * P.win * V) {
            flags = 2;
          } else {
            head_sid = s;
            head_val = fold_acc();
            head_cover = seg_end > r1;
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] = R::identity();
            flags = 1 | (head_cover ? 2 : 0);
          }
#pragma unroll
          for (int u = 0; u < U; ++u) cur[u] = nxt[u];
        } else {
          r0 = P.begin(wi);
          r1 = P.end(wi);
          seek(r0);
          head_sid = -1;
          tail_sid = -1;
          head_cover = false;
          if (wi == 0 && P.A > P.lo) consume_scalar(P.lo, P.A);
          if (vb < P.nvec) {
            const int64_t nv = min(P.win, P.nvec - vb);
            const int64_t P0 = P.A + vb * V;
            A vals[K];
            if (nv == P.win) {
#pragma unroll
              for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < V; ++e) vals[u * V + e] = R::convert(lane_elem<T>(cur[u], e));
            } else {
#pragma unroll
              for (int u = 0; u < U; ++u) {
                const bool ok = (u * 64 + lane) < nv;
#pragma unroll
                for (int e = 0; e < V; ++e)
                  vals[u * V + e] = ok ? R::convert(lane_elem<T>(cur[u], e)) : R::identity();
              }
            }
            consume(vals, rel_vec, P0, P0 + nv * V);
          }
          if (wi == P.nw - 1) {
            const int64_t t0 = P.A + P.nvec * V;
            if (t0 < P.hi) consume_scalar(t0, P.hi);
          }
          // The segment the window ends in.  If it also reaches this
          // wavefront's next window, its piece stays in the accumulators and
          // is reported later (every window between belongs to it); it is
          // reported no later than the window before it ends, so the join
          // always has it in time.
          if (wn < wlast && seg_end > P.begin(wn)) {
            if (seg_begin >= r0) {  // it starts here: restart the join's running piece
              tail_sid = s;
              tail_val = R::identity();
            } else {
              head_cover = true;  // the window lies inside it: nothing to join
            }
          } else {
            emit(s, fold_acc(), seg_begin, seg_end);
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] = R::identity();
          }
          flags = (head_sid >= 0 ? 1 : 0) | (head_cover ? 2 : 0) | (tail_sid >= 0 ? 4 : 0);
#pragma unroll
          for (int u = 0; u < U; ++u) cur[u] = nxt[u];
        }
      }
      if (lane == 0) {  // the join reads a piece only where its flag is set
        const int e = rr * WB + wib;
        e_flags[b][e] = flags;
        if (flags & 1) {
          e_hsid[b][e] = head_sid;
          e_hval[b][e] = head_val;
        }
        if (flags & 4) {
          e_tsid[b][e] = tail_sid;
          e_tval[b][e] = tail_val;
        }
      }
    }
    __syncthreads();
    if (wib == 0)
      for (int c = 0; c < NE; c += 64) join(b, c);
  }
  // The piece still running at the work-group's end belongs to a segment
  // that runs past it.
  if (wib == 0 && jsid >= 0) block_emit(jsid, jrun.v, jbefore, false);
  fill_empty();
}

template <class R, int U, bool NT>
hipError_t launch_seg(const void* x, const int64_t* offsets, int64_t nseg, void* out,
                      const Scratch& ws, const Launch& l, hipStream_t s) {
  hipLaunchKernelGGL((segmented_kernel<R, U, NT>), dim3(l.grid), dim3(l.block), 0, s,
                     (const typename R::T*)x, offsets, nseg, (typename R::Out*)out,
                     ws.carry, ws.counters, ws.ticket + 1);
  return hipGetLastError();
}

template <class R, bool NT> SegFn seg_pick_unroll(int unroll) {
  switch (unroll) {
    case 2: return launch_seg<R, 2, NT>;
    case 4: return launch_seg<R, 4, NT>;
    case 8: return launch_seg<R, 8, NT>;
  }
  return nullptr;
}

template <class R> SegFn seg_pick(int unroll, bool nt) {
  return nt ? seg_pick_unroll<R, true>(unroll) : seg_pick_unroll<R, false>(unroll);
}

}  // namespace rd
