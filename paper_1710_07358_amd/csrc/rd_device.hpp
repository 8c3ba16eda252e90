// rd_device.hpp -- device building blocks of the gfx950 reduction kernels.
//
// * Reduction traits R: storage type T, accumulator Acc, neutral element,
//   combiner, conversion of a stored element, finalisation to the output.
//   (Section 1.1: an associative combiner with a neutral element.)
// * Cross-lane wavefront reduction with DPP (the register-to-register
//   exchange idea of Section 2.2, done with CDNA's data-parallel primitives:
//   quad permutes, row mirrors and row broadcasts; no LDS, no barrier).
// * Work-group stage: one LDS slot per wavefront and a single barrier.  The
//   barrier-free LDS tree of Section 3 is only safe inside one wavefront, so
//   the cross-wavefront step keeps one barrier.
// * Grid stage (stage 2 of Section 2.3, done in the same launch): each
//   work-group publishes one partial, and the last one to arrive at a
//   counter folds them in index order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rd {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

enum class Op { Sum, Prod, Min, Max, And, Or, Xor };

struct dd { double hi, lo; };  // double-double value hi + lo, |lo| <= ulp(hi)/2

// ------------------------------------------------------------------ traits

template <Op O, class A> struct Combiner;

// 32-bit unsigned: + and x wrap modulo 2^32; bitwise ops; unsigned min/max.
template <Op O> struct Combiner<O, uint32_t> {
  static __device__ __forceinline__ uint32_t identity() {
    if constexpr (O == Op::Sum || O == Op::Or || O == Op::Xor || O == Op::Max) return 0u;
    else if constexpr (O == Op::Prod) return 1u;
    else return 0xFFFFFFFFu;  // And, Min
  }
  static __device__ __forceinline__ uint32_t apply(uint32_t a, uint32_t b) {
    if constexpr (O == Op::Sum) return a + b;
    else if constexpr (O == Op::Prod) return a * b;
    else if constexpr (O == Op::Min) return a < b ? a : b;
    else if constexpr (O == Op::Max) return a > b ? a : b;
    else if constexpr (O == Op::And) return a & b;
    else if constexpr (O == Op::Or) return a | b;
    else return a ^ b;
  }
};

template <Op O> struct Combiner<O, int32_t> {  // signed min/max only
  static_assert(O == Op::Min || O == Op::Max, "signed accumulators serve min/max");
  static __device__ __forceinline__ int32_t identity() {
    return O == Op::Min ? (int32_t)0x7FFFFFFF : (int32_t)0x80000000;
  }
  static __device__ __forceinline__ int32_t apply(int32_t a, int32_t b) {
    if constexpr (O == Op::Min) return a < b ? a : b;
    else return a > b ? a : b;
  }
};

// 64-bit unsigned: + and x wrap modulo 2^64; bitwise ops (also the bits of
// float64 data); unsigned min/max.
template <Op O> struct Combiner<O, uint64_t> {
  static __device__ __forceinline__ uint64_t identity() {
    if constexpr (O == Op::Sum || O == Op::Or || O == Op::Xor || O == Op::Max) return 0ull;
    else if constexpr (O == Op::Prod) return 1ull;
    else return ~0ull;  // And, Min
  }
  static __device__ __forceinline__ uint64_t apply(uint64_t a, uint64_t b) {
    if constexpr (O == Op::Sum) return a + b;
    else if constexpr (O == Op::Prod) return a * b;
    else if constexpr (O == Op::Min) return a < b ? a : b;
    else if constexpr (O == Op::Max) return a > b ? a : b;
    else if constexpr (O == Op::And) return a & b;
    else if constexpr (O == Op::Or) return a | b;
    else return a ^ b;
  }
};

template <Op O> struct Combiner<O, int64_t> {  // signed 64-bit min/max only
  static_assert(O == Op::Min || O == Op::Max, "signed accumulators serve min/max");
  static __device__ __forceinline__ int64_t identity() {
    return O == Op::Min ? (int64_t)0x7FFFFFFFFFFFFFFFll : (int64_t)(-0x7FFFFFFFFFFFFFFFll - 1);
  }
  static __device__ __forceinline__ int64_t apply(int64_t a, int64_t b) {
    if constexpr (O == Op::Min) return a < b ? a : b;
    else return a > b ? a : b;
  }
};

// Floats: IEEE arithmetic for +/x; IEEE 754-2019 minimum/maximum (NaN wins,
// -0 < +0), which gfx950 executes as v_minimum3/v_maximum3 for binary32.
template <Op O, class F> struct FloatCombiner {
  static_assert(O == Op::Sum || O == Op::Prod || O == Op::Min || O == Op::Max, "float op");
  static __device__ __forceinline__ F identity() {
    if constexpr (O == Op::Sum) return F(0);
    else if constexpr (O == Op::Prod) return F(1);
    else if constexpr (O == Op::Min) return __builtin_inff();
    else return -__builtin_inff();
  }
  static __device__ __forceinline__ F apply(F a, F b) {
    if constexpr (O == Op::Sum) return a + b;
    else if constexpr (O == Op::Prod) return a * b;
    else if constexpr (O == Op::Min) return __builtin_elementwise_minimum(a, b);
    else return __builtin_elementwise_maximum(a, b);
  }
};
template <Op O> struct Combiner<O, float> : FloatCombiner<O, float> {};
template <Op O> struct Combiner<O, double> : FloatCombiner<O, double> {};

// Storage kinds: how a stored element becomes an accumulator value and how
// the final accumulator becomes the output element.
enum class Store { U32, I32, U64, I64, F32, F64, F16, BF16, U16 };

template <Store S> struct Stored;
template <> struct Stored<Store::U32> { using T = uint32_t; };
template <> struct Stored<Store::I32> { using T = int32_t; };
template <> struct Stored<Store::U64> { using T = uint64_t; };
template <> struct Stored<Store::I64> { using T = int64_t; };
template <> struct Stored<Store::F32> { using T = float; };
template <> struct Stored<Store::F64> { using T = double; };
template <> struct Stored<Store::F16> { using T = uint16_t; };
template <> struct Stored<Store::BF16> { using T = uint16_t; };
template <> struct Stored<Store::U16> { using T = uint16_t; };

__device__ __forceinline__ float f16_to_f32(uint16_t h) {
  return (float)__builtin_bit_cast(_Float16, h);  // exact (v_cvt_f32_f16)
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);  // exact
}

// Full reduction description: storage S, op O.
template <Store S, Op O> struct Red {
  using T = typename Stored<S>::T;
  static constexpr bool half = (S == Store::F16 || S == Store::BF16);
  // accumulator type.  Float products accumulate in float64: a float32
  // product of factors near 1 hovers around 1.0, where round-to-nearest
  // ties are broken one way by the tiny second-order term, so float32
  // accumulation drifts linearly in n (about 6% at n = 2^28).
  using Acc = typename std::conditional<
      (S == Store::F32 || half) && O == Op::Prod, double,
      typename std::conditional<
          S == Store::F32 || half, float,
          typename std::conditional<S == Store::F64, double,
                                    typename std::conditional<S == Store::U16, uint32_t, T>::type>::type>::type>::type;
  // output element type
  using Out = typename std::conditional<
      half && (O == Op::Min || O == Op::Max), uint16_t,
      typename std::conditional<S == Store::U16, uint16_t,
                                typename std::conditional<(S == Store::F32 || half) && O == Op::Prod, float,
                                                          Acc>::type>::type>::type;
  using C = Combiner<O, Acc>;

  static __device__ __forceinline__ Acc identity() { return C::identity(); }
  static __device__ __forceinline__ Acc apply(Acc a, Acc b) { return C::apply(a, b); }
  static __device__ __forceinline__ Acc convert(T v) {
    if constexpr (S == Store::F16) return (Acc)f16_to_f32(v);
    else if constexpr (S == Store::BF16) return (Acc)bf16_to_f32(v);
    else if constexpr (S == Store::U16) return (uint32_t)v;  // upper half ignored by finalize
    else return v;
  }
  static __device__ __forceinline__ Out finalize(Acc a) {
    if constexpr (S == Store::F16 && (O == Op::Min || O == Op::Max))
      return __builtin_bit_cast(uint16_t, (_Float16)a);  // exact: a is a stored binary16 value
    else if constexpr (S == Store::BF16 && (O == Op::Min || O == Op::Max))
      return (uint16_t)(__builtin_bit_cast(uint32_t, a) >> 16);  // exact: low half is zero
    else if constexpr (S == Store::U16) return (uint16_t)a;
    else return (Out)a;  // float64 product -> float32: one rounding
  }
};

// ------------------------------------------------------------------ vector loads

// One 16-byte load per work-item: global_load_dwordx4, optionally non-temporal.
template <bool NT> __device__ __forceinline__ u32x4 load16(const u32x4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// Element e of a 16-byte vector holding 16/sizeof(T) elements of T.
// (The element is copied to a scalar before the bit cast: clang reads element
// 0 when __builtin_bit_cast is applied to a vector-element lvalue directly.)
template <class T> __device__ __forceinline__ T lane_elem(const u32x4& v, int e) {
  if constexpr (sizeof(T) == 4) {
    const uint32_t w = v[e];
    return __builtin_bit_cast(T, w);
  } else if constexpr (sizeof(T) == 8) {
    uint64_t b = (uint64_t)v[2 * e] | ((uint64_t)v[2 * e + 1] << 32);
    return __builtin_bit_cast(T, b);
  } else {
    const uint32_t w = v[e >> 1];
    const uint16_t h = (uint16_t)((e & 1) ? (w >> 16) : (w & 0xFFFFu));
    return __builtin_bit_cast(T, h);
  }
}

// ------------------------------------------------------------------ cross-lane

// dpp<ctrl,row_mask,bank_mask>(v, fill): v from the DPP source lane; lanes
// outside row_mask/bank_mask (or without a valid source) receive `fill`.
template <int CTRL, int ROWS, int BANKS>
__device__ __forceinline__ uint32_t dpp32(uint32_t v, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, CTRL, ROWS, BANKS, false);
}

template <int CTRL, int ROWS, int BANKS = 0xF, class A> __device__ __forceinline__ A dpp(A v, A fill) {
  if constexpr (sizeof(A) == 4) {
    return __builtin_bit_cast(A, dpp32<CTRL, ROWS, BANKS>(__builtin_bit_cast(uint32_t, v),
                                                          __builtin_bit_cast(uint32_t, fill)));
  } else if constexpr (sizeof(A) == 8) {
    uint64_t b = __builtin_bit_cast(uint64_t, v), f = __builtin_bit_cast(uint64_t, fill);
    uint32_t lo = dpp32<CTRL, ROWS, BANKS>((uint32_t)b, (uint32_t)f);
    uint32_t hi = dpp32<CTRL, ROWS, BANKS>((uint32_t)(b >> 32), (uint32_t)(f >> 32));
    return __builtin_bit_cast(A, (uint64_t)lo | ((uint64_t)hi << 32));
  } else {
    static_assert(sizeof(A) == 16, "dpp on 4, 8 or 16 bytes");
    struct W { uint64_t a, b; };
    W w = __builtin_bit_cast(W, v), f = __builtin_bit_cast(W, fill);
    W r;
    r.a = dpp<CTRL, ROWS, BANKS>(w.a, f.a);
    r.b = dpp<CTRL, ROWS, BANKS>(w.b, f.b);
    return __builtin_bit_cast(A, r);
  }
}

template <class A> __device__ __forceinline__ A readlane(A v, int lane) {
  if constexpr (sizeof(A) == 4) {
    return __builtin_bit_cast(A, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else if constexpr (sizeof(A) == 8) {
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(A, (uint64_t)lo | ((uint64_t)hi << 32));
  } else {
    struct W { uint64_t a, b; };
    W w = __builtin_bit_cast(W, v);
    w.a = readlane(w.a, lane);
    w.b = readlane(w.b, lane);
    return __builtin_bit_cast(A, w);
  }
}

// Reduce the 64 lanes of a wavefront; the result is returned to every lane
// (wavefront-uniform).  Fixed combining order, so float results are
// deterministic.  Combine: a binary functor (a, b) -> a (+) b.
template <class A, class Combine>
__device__ __forceinline__ A wave_reduce(A v, A id, Combine comb) {
  v = comb(v, dpp<0xB1, 0xF>(v, id));   // quad_perm [1,0,3,2]: pairs
  v = comb(v, dpp<0x4E, 0xF>(v, id));   // quad_perm [2,3,0,1]: quads
  v = comb(v, dpp<0x141, 0xF>(v, id));  // row_half_mirror: groups of 8
  v = comb(v, dpp<0x140, 0xF>(v, id));  // row_mirror: rows of 16
  v = comb(v, dpp<0x142, 0xA>(v, id));  // row_bcast:15 into rows 1, 3
  v = comb(v, dpp<0x143, 0xC>(v, id));  // row_bcast:31 into rows 2, 3
  return readlane(v, 63);               // lane 63 holds all 64 lanes
}

template <class R> __device__ __forceinline__ typename R::Acc wave_reduce_r(typename R::Acc v) {
  return wave_reduce(v, R::identity(),
                     [](typename R::Acc a, typename R::Acc b) { return R::apply(a, b); });
}

// Work-group reduction; the result is valid in every lane of wavefront 0.
// lds must hold blockDim.x/64 accumulators.  Ends with the block converged.
template <class A, class Combine>
__device__ __forceinline__ A block_reduce(A v, A id, Combine comb, A* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  v = wave_reduce(v, id, comb);
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  A r = id;
  if (wave == 0) {
    r = lane < nwaves ? lds[lane] : id;
    r = wave_reduce(r, id, comb);
  }
  return r;
}

// Inclusive scan over the 64 lanes (lane i gets v0 (+) ... (+) vi), fixed
// order: three shifted combines of the original value give windows of four,
// then row_shr:4 and row_shr:8 complete each row of 16, and two row
// broadcasts carry rows into the rows after them.
template <class A, class Combine>
__device__ __forceinline__ A wave_scan_incl(A v, A id, Combine comb) {
  A r = comb(v, dpp<0x111, 0xF>(v, id));  // row_shr:1
  r = comb(r, dpp<0x112, 0xF>(v, id));    // row_shr:2 (of the original)
  r = comb(r, dpp<0x113, 0xF>(v, id));    // row_shr:3 (of the original)
  r = comb(r, dpp<0x114, 0xF, 0xE>(r, id));  // row_shr:4 into lanes 4..15 of each row
  r = comb(r, dpp<0x118, 0xF, 0xC>(r, id));  // row_shr:8 into lanes 8..15
  r = comb(r, dpp<0x142, 0xA>(r, id));       // row_bcast:15 into rows 1, 3
  r = comb(r, dpp<0x143, 0xC>(r, id));       // row_bcast:31 into rows 2, 3
  return r;
}

// Exclusive scan: the inclusive scan shifted one lane up (wave_shr:1).
template <class A> __device__ __forceinline__ A wave_shift_up(A incl, A id) {
  return dpp<0x138, 0xF>(incl, id);
}

// Value of lane 63 - lane (full reversal of the wavefront, via ds_bpermute).
__device__ __forceinline__ float wave_reverse(float v) {
  const int lane = threadIdx.x & 63;
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((63 - lane) << 2, __builtin_bit_cast(int, v)));
}

// ------------------------------------------------------------------ grid stage

// Publishing a value to the work-group that finishes the reduction.  Each
// 32-bit piece of the value travels in its own 64-bit agent-scope atomic word
// next to a nonzero tag, so a reader that sees the tag sees this launch's
// piece: no ordering between different words is needed, hence no agent-scope
// release/acquire fences (on gfx950 those write back and invalidate the whole
// L2 of the XCD -- about 20 us per launch when every work-group does it).
// The reader clears the words after use, which re-arms the slot for the next
// launch or graph replay.
constexpr uint64_t kTag = 1ull << 32;
constexpr int kMaxSpin = 1 << 20;  // bounded wait; a correct launch never comes close

template <class A> __device__ __forceinline__ void publish(uint64_t* slot, A v) {
  struct P { uint32_t w[sizeof(A) / 4]; };
  const P p = __builtin_bit_cast(P, v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(A) / 4); ++i)
    __hip_atomic_store(slot + i, kTag | (uint64_t)p.w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every word of the slot carries the tag, clear it, return the
// value.  A wait that runs out (impossible unless the launch is broken) sets
// *status and returns what the words hold.
template <class A> __device__ __forceinline__ A collect(uint64_t* slot, unsigned* status) {
  struct P { uint32_t w[sizeof(A) / 4]; };
  P p;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(A) / 4); ++i) {
    uint64_t word = __hip_atomic_load(slot + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int spin = 0; !(word & kTag) && spin < kMaxSpin; ++spin) {
      __builtin_amdgcn_s_sleep(2);
      word = __hip_atomic_load(slot + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!(word & kTag)) __hip_atomic_fetch_or(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    p.w[i] = (uint32_t)word;
    __hip_atomic_store(slot + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return __builtin_bit_cast(A, p);
}

// Count this work-group in and learn whether it is the last of nblocks.
// The counter only elects the finisher; the data arrive through publish /
// collect, so a relaxed agent-scope increment is enough.  The finisher
// re-zeroes the counter for the next launch.
__device__ __forceinline__ bool arrive_last(unsigned* ticket, unsigned nblocks, int* lds_flag) {
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool last = (prev == nblocks - 1);
    if (last) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *lds_flag = last ? 1 : 0;
  }
  __syncthreads();
  return *lds_flag != 0;
}

// Words of one published slot for accumulator type A.
template <class A> constexpr int slot_words() { return (int)(sizeof(A) / 4); }

// ------------------------------------------------------------------ double-double

// Error-free sum of two doubles (Knuth's TwoSum, branch-free).
__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return dd{s, e};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  double lo = s.lo + (a.lo + b.lo);
  double hi = s.hi + lo;
  return dd{hi, lo - (hi - s.hi)};
}

}  // namespace rd
