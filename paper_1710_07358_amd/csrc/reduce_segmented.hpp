// reduce_segmented.hpp -- many segments, one persistent launch (gfx950).
//
// out[s] = x[offsets[s]] (+) ... (+) x[offsets[s+1]-1].
//
// Persistent threads suit irregular work (Section 2.5), so the launch holds a
// fixed grid and the work is split by elements, not by segments: the range
// [offsets[0], offsets[nseg]) is cut into equal, 16-byte-aligned pieces, one
// per wavefront.  A wavefront streams its piece in windows of 64 x U
// sixteen-byte loads (coalesced, as in the plain kernel) while tracking the
// segment it is in (wavefront-uniform state plus a register cache of 64
// offsets).  A window inside one segment is folded straight into the private
// accumulators; a window that crosses segment ends is folded one segment at
// a time with per-element selects (never a multiply-by-flag, Section 3).
//
// A segment wholly inside one wavefront's piece is written directly.  The
// pieces of a segment that crosses pieces are combined first inside each
// work-group (in wavefront order, through LDS); a segment that crosses
// work-groups leaves one partial per work-group, each work-group bumps a
// counter owned by the segment's first work-group, and the one that
// completes the count folds the partials in work-group order and writes the
// result.  The fold order does not depend on arrival order, so the result is
// deterministic.  Empty segments are written with the neutral
// element by a grid-stride pass at the end.
#pragma once

#include "rd_device.hpp"
#include "rd_internal.hpp"

namespace rd {

namespace {

__device__ __forceinline__ int64_t rl64(int64_t v, int lane) { return readlane(v, lane); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Partition of [lo, hi) into wavefront pieces: an unaligned head (< V
// elements, piece 0), nvec 16-byte vectors (per vectors per piece) and a
// ragged tail (< V elements).  Pieces 0..wt are non-empty; the tail goes to
// wt, the last piece holding vectors, so every wavefront between two that a
// segment touches has work and reports its part of that segment.
struct Partition {
  int64_t lo, hi, A, nvec, per, wt;
  int V;
  __device__ int64_t r0(int64_t w) const { return w == 0 ? lo : A + min(w * per, nvec) * V; }
  __device__ int64_t r1(int64_t w) const {
    return w == wt ? hi : (w > wt ? r0(w) : A + min((w + 1) * per, nvec) * V);
  }
  __device__ int64_t wave_of(int64_t pos) const {
    if (pos < A) return 0;
    const int64_t vec = (pos - A) / V;
    if (vec >= nvec) return wt;
    return min(vec / per, wt);
  }
};

}  // namespace

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
  constexpr int V = 16 / (int)sizeof(T);
  constexpr int K = U * V;  // elements per lane per window
  const int lane = threadIdx.x & 63;

  // Empty segments get the neutral element (no other path writes them:
  // the walk over segments skips them).  Done last, so its loads do not
  // delay the first data loads.
  const auto fill_empty = [&]() {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nseg; s += stride)
      if (offsets[s + 1] <= offsets[s]) out[s] = R::finalize(R::identity());
  };

  // ---- this wavefront's piece
  Partition P;
  const int64_t W = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  P.lo = offsets[0];
  P.hi = offsets[nseg];
  if (P.hi <= P.lo) {
    fill_empty();
    return;
  }
  P.V = V;
  {
    const uintptr_t a = (uintptr_t)(x + P.lo);
    int64_t head = (int64_t)(((16u - (unsigned)(a & 15u)) & 15u) / sizeof(T));
    P.A = min(P.lo + head, P.hi);
    P.nvec = (P.hi - P.A) / V;
    const int64_t win = 64 * U;
    int64_t per = (P.nvec + W - 1) / W;
    per = (per + win - 1) / win * win;
    P.per = per > 0 ? per : win;
    P.wt = P.nvec > 0 ? (P.nvec - 1) / P.per : 0;
  }
  const int64_t r0 = P.r0(w), r1 = P.r1(w);
  const bool work = r0 < r1;  // pieces past the last one are empty
  // Pieces of segments that cross this wavefront's range: at most one that
  // began before r0 (head; it may also run past r1: covering) and one that
  // runs past r1 (tail).  They are combined per work-group at the end.
  int64_t head_sid = -1, tail_sid = -1;
  A head_val = R::identity(), tail_val = R::identity();
  bool head_cover = false;
  if (work) {

    // The first window's loads go out before the segment search, so the
    // search's dependent offset loads overlap them.
    const int64_t v0 = min(w * P.per, P.nvec), v1 = min((w + 1) * P.per, P.nvec);
    const u32x4* xv = (const u32x4*)(x + P.A);
    // Windows of 64 x U vectors, software-pipelined: the next window's loads
    // are issued before the current one is folded, so segment bookkeeping at
    // boundaries overlaps memory latency.  Vectors at or past v1 are not read.
    auto load_window = [&](int64_t vb, u32x4 (&raw)[U]) {
      const int64_t nv = min((int64_t)(64 * U), v1 - vb);
      if (nv == 64 * U) {
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
    u32x4 cur[U], nxt[U];
    if (v0 < v1) load_window(v0, cur);

    // ---- segment containing r0: largest s < nseg with offsets[s] <= r0 (64-ary search)
    int64_t s;
    {
      int64_t a = 0, b = nseg - 1;  // answer in [a, b]; offsets[a] <= r0 holds
      while (b - a >= 64) {
        const int64_t step = (b - a + 63) / 64;
        const int64_t idx = min(a + (int64_t)lane * step, b);
        const uint64_t m = ballot(offsets[idx] <= r0);  // prefix of lanes (offsets sorted)
        const int k = __builtin_popcountll(m) - 1;      // >= 0 since lane 0 holds offsets[a]
        const int64_t na = min(a + (int64_t)k * step, b);  // probes past b were clamped to b
        b = min(na + step - 1, b);
        a = na;
      }
      const int64_t idx = min(a + (int64_t)lane, b);
      const uint64_t m = ballot(a + lane <= b && offsets[idx] <= r0);
      s = a + __builtin_popcountll(m) - 1;
    }

    // Register cache of offsets[cbase .. cbase+63] (indices clamped to nseg).
    int64_t cbase = s + 1;
    int64_t cache = offsets[min(cbase + lane, nseg)];
    auto offset_at = [&](int64_t j) -> int64_t {  // j in [s+1, nseg]; wavefront-uniform
      if (j < cbase || j >= cbase + 64) {
        cbase = j;
        cache = offsets[min(cbase + lane, nseg)];
      }
      return rl64(cache, (int)(j - cbase));
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

    int64_t seg_begin = offsets[s];
    int64_t seg_end = offset_at(s + 1);

    A acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = R::identity();

    auto fold_acc = [&]() -> A {
      A v = acc[0];
#pragma unroll
      for (int k = 1; k < K; ++k) v = R::apply(v, acc[k]);
      return wave_reduce_r<R>(v);
    };

    // Piece of segment `sid` covering [sb, se) from this wavefront's view:
    // written at once when the segment lies inside the range, else kept for
    // the work-group stage.
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
    // segments they belong to.  Window = [P0, wend).
    auto consume = [&](const A (&vals)[K], auto rel, int64_t P0, int64_t wend) {
      int64_t consumed = P0;
      while (seg_end < wend) {
        const int32_t from = (int32_t)(consumed - P0), bound = (int32_t)(seg_end - P0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int32_t q = rel(k);
          const A v = (q >= from && q < bound) ? vals[k] : R::identity();
          acc[k] = R::apply(acc[k], v);
        }
        emit(s, fold_acc(), seg_begin, seg_end);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = R::identity();
        consumed = seg_end;
        s = next_segment(s, seg_end);
        seg_begin = consumed;
        seg_end = offset_at(s + 1);
      }
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

    // Scalar piece (head or tail): one element per lane, positions P0 + lane.
    auto consume_scalar = [&](int64_t P0, int64_t wend) {
      A vals[K];
#pragma unroll
      for (int k = 0; k < K; ++k) vals[k] = R::identity();
      if (P0 + lane < wend) vals[0] = R::convert(x[P0 + lane]);
      consume(vals, [&](int k) { return k == 0 ? (int32_t)lane : (int32_t)0x7FFFFFFF; }, P0, wend);
    };

    if (w == 0 && P.A > P.lo) consume_scalar(P.lo, P.A);

    auto rel_vec = [&](int k) { return (int32_t)(((k / V) * 64 + lane) * V + (k % V)); };
    for (int64_t vb = v0; vb < v1; vb += 64 * U) {
      const int64_t vn = vb + 64 * U;
      if (vn < v1) load_window(vn, nxt);
      const int64_t nv = min((int64_t)(64 * U), v1 - vb);
      const int64_t P0 = P.A + vb * V;
      A vals[K];
      if (nv == 64 * U) {
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
#pragma unroll
      for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }

    if (w == P.wt) {
      const int64_t t0 = P.A + P.nvec * V;
      if (t0 < P.hi) consume_scalar(t0, P.hi);
    }

    // The last segment this wavefront touched.
    emit(s, fold_acc(), seg_begin, seg_end);
  }  // work

  // ---- work-group stage: walk the wavefronts in order, finish segments that
  // cross wavefronts inside this work-group, and publish at most two pieces
  // per work-group (one for a segment that began before the work-group, one
  // for a segment that runs past it).  Each crossing segment counts in at
  // its first work-group; the work-group completing the count folds the
  // pieces in work-group order (deterministic).
  __shared__ int64_t lds_hsid[16], lds_tsid[16];
  __shared__ A lds_hval[16], lds_tval[16];
  __shared__ int lds_hcov[16];
  const int wib = threadIdx.x >> 6, WB = blockDim.x >> 6;
  if (lane == 0) {
    lds_hsid[wib] = head_sid;
    lds_hval[wib] = head_val;
    lds_hcov[wib] = head_cover ? 1 : 0;
    lds_tsid[wib] = tail_sid;
    lds_tval[wib] = tail_val;
  }
  __syncthreads();
  if (wib == 0) {
    constexpr int SW = slot_words<A>();
    static_assert(SW <= kCarryWords, "carry slot too small");
    const int64_t blk = blockIdx.x;
    auto block_of = [&](int64_t pos) { return P.wave_of(pos) / WB; };
    // A crossing segment's piece from this work-group; `before`: the segment
    // began before the work-group.
    auto block_emit = [&](int64_t sid, A piece, bool before, bool ends_here) {
      if (!before && ends_here) {
        if (lane == 0) out[sid] = R::finalize(piece);
        return;
      }
      const int64_t bf = block_of(offsets[sid]), bl = block_of(offsets[sid + 1] - 1);
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
    int64_t run_sid = -1;
    A run_val = R::identity();
    bool run_before = false;
    for (int i = 0; i < WB; ++i) {
      const int64_t hs = lds_hsid[i];
      if (hs >= 0) {
        if (run_sid < 0) {  // only wavefront 0: the segment began before the work-group
          run_sid = hs;
          run_val = lds_hval[i];
          run_before = true;
        } else {
          run_val = R::apply(run_val, lds_hval[i]);
        }
        if (!lds_hcov[i]) {
          block_emit(run_sid, run_val, run_before, true);
          run_sid = -1;
        }
      }
      const int64_t ts = lds_tsid[i];
      if (ts >= 0) {
        run_sid = ts;
        run_val = lds_tval[i];
        run_before = false;
      }
    }
    if (run_sid >= 0) block_emit(run_sid, run_val, run_before, false);
  }
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
