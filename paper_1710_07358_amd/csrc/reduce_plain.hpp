// reduce_plain.hpp -- one-launch reduction of a device array (gfx950).
//
// Stage-1 step 1 of Section 3 (persistent work-items, global-memory loop
// unrolled F times) becomes: every work-item issues U independent 16-byte
// loads per step (global_load_dwordx4; 4 x 32-bit, 2 x 64-bit or 8 x 16-bit
// elements), adjacent work-items reading adjacent 16-byte words, and folds
// them into U x V private accumulators.  The grid is persistent (Section
// 2.5): a fixed number of work-groups walks the array in chunks of
// block x U vectors.  Out-of-range work never reads memory: the unaligned
// head and ragged tail are handled by separate guarded element loads, so
// no multiply-by-0/1 mask (Section 3) is needed and every op keeps its own
// neutral element.  Step 3 (per-group reduction) is the DPP wavefront stage
// plus one LDS barrier, and stage 2 (Section 2.3) is the last-block-done
// fold in the same launch.
#pragma once

#include "rd_device.hpp"
#include "rd_internal.hpp"

namespace rd {

// The chunks (of block x U vectors) a work-group visits: first, first + step,
// ... below end.  Layout 0 is the grid-stride order of Section 2.3; layout 1
// renumbers work-groups so that those dispatched to one XCD (work-groups are
// dealt round-robin to the 8 XCDs) take adjacent chunks; layout 2 gives each
// work-group one contiguous run.
struct ChunkWalk {
  int64_t first, end, step;
};
__device__ __forceinline__ ChunkWalk chunk_walk(int layout, int64_t nchunks) {
  const int64_t G = gridDim.x, b = blockIdx.x;
  if (layout == 2) {
    const int64_t per = nchunks / G, extra = nchunks % G;
    const int64_t first = b * per + (b < extra ? b : extra);
    return ChunkWalk{first, first + per + (b < extra ? 1 : 0), 1};
  }
  int64_t lb = b;
  if (layout == 1 && (G & 7) == 0) lb = (b & 7) * (G >> 3) + (b >> 3);
  return ChunkWalk{lb, nchunks, G};
}

template <class R, int U, bool NT>
__global__ __launch_bounds__(1024) void reduce_kernel(const typename R::T* __restrict__ x,
                                                      int64_t n,
                                                      uint64_t* __restrict__ partial,
                                                      unsigned* __restrict__ ticket,
                                                      typename R::Out* __restrict__ out, int layout,
                                                      int probe) {
  using T = typename R::T;
  using A = typename R::Acc;
  constexpr int V = 16 / (int)sizeof(T);
  __shared__ A lds[16];
  __shared__ int last_flag;

  const int tid = threadIdx.x;
  const int64_t B = blockDim.x, G = gridDim.x;

  // Split x into an unaligned head (< V elements), 16-byte vectors, and a tail.
  const uintptr_t addr = (uintptr_t)x;
  int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) / sizeof(T));
  if (head > n) head = n;
  const u32x4* xv = (const u32x4*)(x + head);
  const int64_t nvec = (n - head) / V;

  A acc[U][V];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < V; ++e) acc[u][e] = R::identity();

  const int64_t step = B * U;  // vectors per chunk
  const int64_t nfull = nvec / step;
  const ChunkWalk walk = chunk_walk(layout, nfull);
  for (int64_t c = walk.first; c < walk.end; c += walk.step) {
    const u32x4* p = xv + c * step + tid;
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load16<NT>(p + u * B);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < V; ++e) acc[u][e] = R::apply(acc[u][e], R::convert(lane_elem<T>(v[u], e)));
  }
  // Remaining vectors (less than one chunk), spread over the whole grid.
  for (int64_t i = nfull * step + blockIdx.x * B + tid; i < nvec; i += G * B) {
    const u32x4 v = load16<NT>(xv + i);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[0][e] = R::apply(acc[0][e], R::convert(lane_elem<T>(v, e)));
  }
  // Unaligned head and ragged tail, one element per work-item.
  const int64_t gtid = blockIdx.x * B + tid;
  const int64_t tail0 = head + nvec * V;
  if (gtid < head) acc[0][0] = R::apply(acc[0][0], R::convert(x[gtid]));
  if (gtid < n - tail0) acc[U - 1][V - 1] = R::apply(acc[U - 1][V - 1], R::convert(x[tail0 + gtid]));

  // Private accumulators -> one value per work-item (fixed order).
  A mine = acc[0][0];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < V; ++e)
      if (u | e) mine = R::apply(mine, acc[u][e]);

  auto comb = [](A a, A b) { return R::apply(a, b); };
  A blk = block_reduce(mine, R::identity(), comb, lds);
  constexpr int SW = slot_words<A>();
  if (tid == 0) publish(partial + blockIdx.x * SW, blk);

  if (arrive_last(ticket, (unsigned)G, &last_flag)) {
    // probe (failure-path test only): also collect slot G, which no work-group
    // publishes, so that one bounded wait runs out and sets the status word.
    A r = R::identity();
    for (int64_t b = tid; b < G + probe; b += B) r = R::apply(r, collect<A>(partial + b * SW, ticket + 1));
    r = block_reduce(r, R::identity(), comb, lds);
    if (tid == 0) *out = R::finalize(r);
  }
}

// Compensated sum: every accumulator slot is an error-free (s, c) pair in
// float32 -- TwoSum keeps the rounding error of each addition exactly, and
// c collects those errors.  Pairs leave the work-item as double-double and
// are merged in float64 (DPP, LDS and the last-block-done fold).
static_assert(sizeof(dd) / 4 <= kPartialWords, "partial slot too small");
// LB: the largest work-group the instantiation serves.  (s, c) pairs double
// the accumulator registers; with LB = 256 the compiler may give a wavefront
// up to 512 VGPRs, so U = 8 and 16 run without spilling.
template <Store S, int U, bool NT, int LB>
__global__ __launch_bounds__(LB) void reduce_compensated_kernel(
    const typename Stored<S>::T* __restrict__ x, int64_t n, uint64_t* __restrict__ partial,
    unsigned* __restrict__ ticket, double* __restrict__ out, int layout) {
#pragma clang fp contract(off)
  using T = typename Stored<S>::T;
  using R = Red<S, Op::Sum>;
  constexpr int V = 16 / (int)sizeof(T);
  __shared__ dd lds[16];
  __shared__ int last_flag;

  const int tid = threadIdx.x;
  const int64_t B = blockDim.x, G = gridDim.x;
  const uintptr_t addr = (uintptr_t)x;
  int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) / sizeof(T));
  if (head > n) head = n;
  const u32x4* xv = (const u32x4*)(x + head);
  const int64_t nvec = (n - head) / V;

  float s[U][V], c[U][V];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < V; ++e) s[u][e] = c[u][e] = 0.0f;

  auto two_sum_into = [](float& sum, float& err, float v) {
    const float t = sum + v;
    const float z = t - sum;
    err += (sum - (t - z)) + (v - z);
    sum = t;
  };

  const int64_t step = B * U;
  const int64_t nfull = nvec / step;
  const ChunkWalk walk = chunk_walk(layout, nfull);
  for (int64_t ch = walk.first; ch < walk.end; ch += walk.step) {
    const u32x4* p = xv + ch * step + tid;
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load16<NT>(p + u * B);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < V; ++e) two_sum_into(s[u][e], c[u][e], R::convert(lane_elem<T>(v[u], e)));
  }
  for (int64_t i = nfull * step + blockIdx.x * B + tid; i < nvec; i += G * B) {
    const u32x4 v = load16<NT>(xv + i);
#pragma unroll
    for (int e = 0; e < V; ++e) two_sum_into(s[0][e], c[0][e], R::convert(lane_elem<T>(v, e)));
  }
  const int64_t gtid = blockIdx.x * B + tid;
  const int64_t tail0 = head + nvec * V;
  if (gtid < head) two_sum_into(s[0][0], c[0][0], R::convert(x[gtid]));
  if (gtid < n - tail0) two_sum_into(s[U - 1][V - 1], c[U - 1][V - 1], R::convert(x[tail0 + gtid]));

  dd mine{0.0, 0.0};
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < V; ++e) mine = dd_add(mine, two_sum((double)s[u][e], (double)c[u][e]));

  auto comb = [](dd a, dd b) { return dd_add(a, b); };
  const dd zero{0.0, 0.0};
  dd blk = block_reduce(mine, zero, comb, lds);
  constexpr int SW = slot_words<dd>();
  if (tid == 0) publish(partial + blockIdx.x * SW, blk);
  if (arrive_last(ticket, (unsigned)G, &last_flag)) {
    dd r = zero;
    for (int64_t b = tid; b < G; b += B) r = dd_add(r, collect<dd>(partial + b * SW, ticket + 1));
    r = block_reduce(r, zero, comb, lds);
    if (tid == 0) *out = r.hi + r.lo;
  }
}

// ------------------------------------------------------------------ launchers

template <class R, int U, bool NT>
hipError_t launch_plain(const void* x, int64_t n, void* out, const Scratch& ws, const Launch& l,
                        hipStream_t s) {
  hipLaunchKernelGGL((reduce_kernel<R, U, NT>), dim3(l.grid), dim3(l.block), 0, s,
                     (const typename R::T*)x, n, ws.partial, ws.ticket,
                     (typename R::Out*)out, l.layout, l.probe ? 1 : 0);
  return hipGetLastError();
}

template <Store S, int U, bool NT>
hipError_t launch_comp(const void* x, int64_t n, void* out, const Scratch& ws, const Launch& l,
                       hipStream_t s) {
  if (l.block <= 256)
    hipLaunchKernelGGL((reduce_compensated_kernel<S, U, NT, 256>), dim3(l.grid), dim3(l.block), 0, s,
                       (const typename Stored<S>::T*)x, n, ws.partial, ws.ticket, (double*)out, l.layout);
  else
    hipLaunchKernelGGL((reduce_compensated_kernel<S, U, NT, 1024>), dim3(l.grid), dim3(l.block), 0, s,
                       (const typename Stored<S>::T*)x, n, ws.partial, ws.ticket, (double*)out, l.layout);
  return hipGetLastError();
}

template <class R, bool NT> PlainFn pick_unroll(int unroll) {
  switch (unroll) {
    case 1: return launch_plain<R, 1, NT>;
    case 2: return launch_plain<R, 2, NT>;
    case 4: return launch_plain<R, 4, NT>;
    case 8: return launch_plain<R, 8, NT>;
    case 16: return launch_plain<R, 16, NT>;
  }
  return nullptr;
}

template <class R> PlainFn pick(int unroll, bool nt) {
  return nt ? pick_unroll<R, true>(unroll) : pick_unroll<R, false>(unroll);
}

template <Store S, bool NT> PlainFn pick_comp_unroll(int unroll) {
  switch (unroll) {
    case 1: return launch_comp<S, 1, NT>;
    case 2: return launch_comp<S, 2, NT>;
    case 4: return launch_comp<S, 4, NT>;
    case 8: return launch_comp<S, 8, NT>;
    case 16: return launch_comp<S, 16, NT>;
  }
  return nullptr;
}

template <Store S> PlainFn pick_comp(int unroll, bool nt) {
  return nt ? pick_comp_unroll<S, true>(unroll) : pick_comp_unroll<S, false>(unroll);
}

}  // namespace rd
