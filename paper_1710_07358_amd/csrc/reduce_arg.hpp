// reduce_arg.hpp -- min/max together with the lowest index attaining it,
// one launch, every dtype (the (value, index) form of the reduction of
// Section 1.1 with min or max as the combiner).
//
// Hot loop (same streaming structure as the plain kernel): each accumulator
// slot keeps the running min/max (IEEE 754-2019 for floats: NaN wins, -0 <
// +0) and the chunk in which its bit pattern last changed -- equal values
// leave it unchanged, so the first occurrence is kept.  Afterwards every
// candidate becomes (score, index): an order-preserving unsigned score (larger
// wins, NaN highest) and its element index (smaller wins on equal scores).
// Candidates combine through DPP, LDS and the tagged grid stage; the last
// work-group reads the winning element back from x, so the returned value is
// exactly the stored one.
#pragma once

#include "reduce_plain.hpp"

namespace rd {

struct ArgCand {
  uint64_t score;
  int64_t idx;  // INT64_MAX: no candidate
};

__device__ __forceinline__ ArgCand arg_better(ArgCand a, ArgCand b) {
  return (a.score > b.score || (a.score == b.score && a.idx < b.idx)) ? a : b;
}

template <Store S> struct ArgTraits;  // Acc: running value; score(): order-preserving key

template <bool MAX> __device__ __forceinline__ uint64_t orient32(uint32_t ukey) {
  return MAX ? (uint64_t)ukey : (uint64_t)(~ukey);
}
template <bool MAX> __device__ __forceinline__ uint64_t orient64(uint64_t ukey) { return MAX ? ukey : ~ukey; }

template <> struct ArgTraits<Store::I32> {
  using Acc = int32_t;
  template <bool MAX> static __device__ __forceinline__ uint64_t score(Acc v) {
    return orient32<MAX>((uint32_t)v ^ 0x80000000u);
  }
};
template <> struct ArgTraits<Store::U32> {
  using Acc = uint32_t;
  template <bool MAX> static __device__ __forceinline__ uint64_t score(Acc v) { return orient32<MAX>(v); }
};
template <> struct ArgTraits<Store::I64> {
  using Acc = int64_t;
  template <bool MAX> static __device__ __forceinline__ uint64_t score(Acc v) {
    return orient64<MAX>((uint64_t)v ^ 0x8000000000000000ull);
  }
};
template <> struct ArgTraits<Store::U64> {
  using Acc = uint64_t;
  template <bool MAX> static __device__ __forceinline__ uint64_t score(Acc v) { return orient64<MAX>(v); }
};
struct ArgFloat32 {
  using Acc = float;
  template <bool MAX> static __device__ __forceinline__ uint64_t score(float v) {
    if (v != v) return ~0ull;  // NaN wins either way
    const uint32_t b = __builtin_bit_cast(uint32_t, v);
    const uint32_t key = b ^ ((uint32_t)((int32_t)b >> 31) & 0x7FFFFFFFu);  // signed order
    return orient32<MAX>(key ^ 0x80000000u) & 0xFFFFFFFFull;
  }
};
template <> struct ArgTraits<Store::F32> : ArgFloat32 {};
template <> struct ArgTraits<Store::F16> : ArgFloat32 {};
template <> struct ArgTraits<Store::BF16> : ArgFloat32 {};
template <> struct ArgTraits<Store::F64> {
  using Acc = double;
  template <bool MAX> static __device__ __forceinline__ uint64_t score(double v) {
    if (v != v) return ~0ull;
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t key = b ^ ((uint64_t)((int64_t)b >> 63) & 0x7FFFFFFFFFFFFFFFull);
    return orient64<MAX>(key ^ 0x8000000000000000ull);
  }
};

template <Store S> __device__ __forceinline__ typename ArgTraits<S>::Acc arg_convert(typename Stored<S>::T v) {
  if constexpr (S == Store::F16) return f16_to_f32(v);
  else if constexpr (S == Store::BF16) return bf16_to_f32(v);
  else return v;
}

template <Store S, bool MAX> __device__ __forceinline__ typename ArgTraits<S>::Acc arg_identity() {
  using A = typename ArgTraits<S>::Acc;
  if constexpr (std::is_floating_point<A>::value) return MAX ? -(A)__builtin_inf() : (A)__builtin_inf();
  else if constexpr (std::is_signed<A>::value)
    return MAX ? (A)((typename std::make_unsigned<A>::type)1 << (8 * sizeof(A) - 1)) : (A)(~((typename std::make_unsigned<A>::type)1 << (8 * sizeof(A) - 1)));
  else return MAX ? (A)0 : (A)~(A)0;
}

// Bits of an accumulator value (for the "did the running extreme change" test).
template <class A> __device__ __forceinline__ auto acc_bits(A v) {
  if constexpr (sizeof(A) == 4) return __builtin_bit_cast(uint32_t, v);
  else return __builtin_bit_cast(uint64_t, v);
}

template <Store S, bool MAX> __device__ __forceinline__ typename ArgTraits<S>::Acc arg_pick(
    typename ArgTraits<S>::Acc a, typename ArgTraits<S>::Acc b) {
  using A = typename ArgTraits<S>::Acc;
  if constexpr (std::is_floating_point<A>::value)
    return MAX ? __builtin_elementwise_maximum(a, b) : __builtin_elementwise_minimum(a, b);
  else return MAX ? (a > b ? a : b) : (a < b ? a : b);
}

template <Store S, bool MAX, int U, bool NT>
__global__ __launch_bounds__(1024) void argreduce_kernel(const typename Stored<S>::T* __restrict__ x, int64_t n,
                                                         uint64_t* __restrict__ partial, unsigned* __restrict__ ticket,
                                                         typename Stored<S>::T* __restrict__ value_out,
                                                         int64_t* __restrict__ index_out, int layout) {
  using T = typename Stored<S>::T;
  using A = typename ArgTraits<S>::Acc;
  using TR = ArgTraits<S>;
  constexpr int V = 16 / (int)sizeof(T);
  __shared__ ArgCand lds[16];
  __shared__ int last_flag;
  const int tid = threadIdx.x;
  const int64_t B = blockDim.x, G = gridDim.x;

  const uintptr_t addr = (uintptr_t)x;
  int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) / sizeof(T));
  if (head > n) head = n;
  const u32x4* xv = (const u32x4*)(x + head);
  const int64_t nvec = (n - head) / V;

  A best[U][V];
  int32_t at[U][V];  // chunk where best last changed, -1: never
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < V; ++e) {
      best[u][e] = arg_identity<S, MAX>();
      at[u][e] = -1;
    }

  const int64_t step = B * U;
  const int64_t nfull = nvec / step;
  const ChunkWalk walk = chunk_walk(layout, nfull);
  // The first chunk seeds every slot with a real element (even one equal to
  // the neutral element, whose bits would not register as a change).
  if (walk.first < walk.end) {
    const int64_t c = walk.first;
    const u32x4* p = xv + c * step + tid;
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load16<NT>(p + u * B);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        best[u][e] = arg_convert<S>(lane_elem<T>(v[u], e));
        at[u][e] = (int32_t)c;
      }
  }
  for (int64_t c = walk.first + walk.step; c < walk.end; c += walk.step) {
    const u32x4* p = xv + c * step + tid;
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load16<NT>(p + u * B);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const A nb = arg_pick<S, MAX>(best[u][e], arg_convert<S>(lane_elem<T>(v[u], e)));
        bool changed = acc_bits(nb) != acc_bits(best[u][e]);
        if constexpr (std::is_floating_point<A>::value) changed = changed && (best[u][e] == best[u][e]);
        at[u][e] = changed ? (int32_t)c : at[u][e];
        best[u][e] = nb;
      }
  }

  // Candidates of this work-item.
  ArgCand mine{0ull, INT64_MAX};
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < V; ++e)
      if (at[u][e] >= 0) {
        const int64_t idx = head + (((int64_t)at[u][e] * step + (int64_t)u * B + tid) * V + e);
        mine = arg_better(mine, ArgCand{TR::template score<MAX>(best[u][e]), idx});
      }
  // Remaining vectors (less than one chunk), the unaligned head and the tail,
  // with their exact indices.
  for (int64_t i = nfull * step + blockIdx.x * B + tid; i < nvec; i += G * B) {
    const u32x4 v = load16<NT>(xv + i);
#pragma unroll
    for (int e = 0; e < V; ++e)
      mine = arg_better(mine, ArgCand{TR::template score<MAX>(arg_convert<S>(lane_elem<T>(v, e))), head + i * V + e});
  }
  const int64_t gtid = blockIdx.x * B + tid;
  const int64_t tail0 = head + nvec * V;
  if (gtid < head) mine = arg_better(mine, ArgCand{TR::template score<MAX>(arg_convert<S>(x[gtid])), gtid});
  if (gtid < n - tail0)
    mine = arg_better(mine, ArgCand{TR::template score<MAX>(arg_convert<S>(x[tail0 + gtid])), tail0 + gtid});

  const ArgCand none{0ull, INT64_MAX};
  auto comb = [](ArgCand a, ArgCand b) { return arg_better(a, b); };
  const ArgCand blk = block_reduce(mine, none, comb, lds);
  constexpr int SW = slot_words<ArgCand>();
  static_assert(SW <= kPartialWords, "partial slot too small");
  if (tid == 0) publish(partial + blockIdx.x * SW, blk);
  if (arrive_last(ticket, (unsigned)G, &last_flag)) {
    ArgCand r = none;
    for (int64_t b = tid; b < G; b += B) r = arg_better(r, collect<ArgCand>(partial + b * SW, ticket + 1));
    r = block_reduce(r, none, comb, lds);
    if (tid == 0) {
      // Every element equal to the neutral element leaves no candidate: the
      // first element then attains the extreme.
      const int64_t idx = (n == 0) ? -1 : (r.idx == INT64_MAX ? 0 : r.idx);
      *index_out = idx;
      if (idx >= 0) {
        *value_out = x[idx];
      } else {
        const A id = arg_identity<S, MAX>();
        if constexpr (S == Store::F16) *value_out = __builtin_bit_cast(uint16_t, (_Float16)id);
        else if constexpr (S == Store::BF16) *value_out = (uint16_t)(__builtin_bit_cast(uint32_t, id) >> 16);
        else *value_out = (T)id;
      }
    }
  }
}

template <Store S, bool MAX, int U, bool NT>
hipError_t launch_arg(const void* x, int64_t n, void* value_out, int64_t* index_out, const Scratch& ws,
                      const Launch& l, hipStream_t s) {
  using T = typename Stored<S>::T;
  hipLaunchKernelGGL((argreduce_kernel<S, MAX, U, NT>), dim3(l.grid), dim3(l.block), 0, s, (const T*)x, n,
                     ws.partial, ws.ticket, (T*)value_out, index_out, l.layout);
  return hipGetLastError();
}

}  // namespace rd
