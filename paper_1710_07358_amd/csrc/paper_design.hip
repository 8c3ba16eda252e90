// paper_design.hip -- the paper's own kernel designs, rebuilt on gfx950 as
// measured baselines for the tuned kernels (sum of int32 or float32 only).
//
// variant 0 -- the two-stage reduction of Section 2.3.  Stage 1 launches as
//   many work-items as the device keeps resident; each folds a strided share
//   of the input (one scalar load per element), the work-group then combines
//   its values in local memory by repeated halving with a barrier after every
//   level, and one value per work-group goes to a partials array.  Stage 2 is
//   a second launch: one work-group reduces the partials the same way.
// variant 1 -- the approach of Section 3.  The global loop is unrolled F
//   times: each work-item takes F consecutive elements per round, rounds
//   strided by the global size times F; the bounds test is folded into the
//   arithmetic instead of a branch (an out-of-range term is 0 times x[0], so
//   nothing past the end is read).  The in-group combine drops the barriers
//   and the divergent branch: every work-item runs the same instructions at
//   every level and a 0/1 factor switches off the upper half's contribution.
//   Without barriers this is only correct when the work-group is a single
//   wavefront, so variant 1 runs 64 work-items per group.  Stage 2 as in
//   variant 0.
#include "rd_device.hpp"
#include "rd_internal.hpp"

namespace rd {

namespace {

// Work-group combine of Section 2.3: `vals` holds blockDim.x values in local
// memory; the live width halves each level (the upper half folds onto the
// lower half), with a barrier between levels.  The result is left in vals[0].
template <class T> __device__ void lds_halving_sum(T* vals) {
  const int lid = threadIdx.x;
  __syncthreads();
  for (int live = blockDim.x; live > 1; live >>= 1) {
    const int half = live >> 1;
    if (lid < half) vals[lid] = vals[lid] + vals[lid + half];
    __syncthreads();
  }
}

template <class T>
__global__ __launch_bounds__(1024) void design_strided_partials(const T* __restrict__ x, int64_t n,
                                                                T* __restrict__ partial) {
  extern __shared__ unsigned char smem[];
  T* vals = (T*)smem;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  T mine = T(0);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) mine = mine + x[i];
  vals[threadIdx.x] = mine;
  lds_halving_sum(vals);
  if (threadIdx.x == 0) partial[blockIdx.x] = vals[0];
}

// Stage 2 (both variants): one work-group folds `count` partials.
template <class T>
__global__ __launch_bounds__(1024) void design_final(const T* __restrict__ partial, int64_t count,
                                                     T* __restrict__ out) {
  extern __shared__ unsigned char smem[];
  T* vals = (T*)smem;
  T mine = T(0);
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) mine = mine + partial[i];
  vals[threadIdx.x] = mine;
  lds_halving_sum(vals);
  if (threadIdx.x == 0) *out = vals[0];
}

// Section 3: F-way unrolled global loop with the algebraic bounds guard, then
// the barrier-free, branch-free combine over one wavefront.  The F terms of a
// round go to F separate running sums (the independent operations unrolling
// exposes), added together once at the end.
template <class T, int F>
__global__ __launch_bounds__(64) void design_unrolled_partials(const T* __restrict__ x, int64_t n,
                                                               T* __restrict__ partial) {
  __shared__ T wave_vals[64];
  const int lid = threadIdx.x;
  const int64_t first = ((int64_t)blockIdx.x * 64 + lid) * F;
  const int64_t round = (int64_t)gridDim.x * 64 * F;
  T run[F];
#pragma unroll
  for (int k = 0; k < F; ++k) run[k] = T(0);
  for (int64_t base = first; base < n; base += round) {
#pragma unroll
    for (int k = 0; k < F; ++k) {
      const int64_t i = base + k;
      const T inside = T(i < n);                 // 1 in range, 0 past the end
      run[k] = run[k] + inside * x[i < n ? i : 0];
    }
  }
  T mine = T(0);
#pragma unroll
  for (int k = 0; k < F; ++k) mine = mine + run[k];
  // One wavefront executes in lockstep, so each level's reads of wave_vals
  // complete before its writes; all 64 lanes run every level, and the upper
  // lanes' sums (reading a wrapped-around neighbour) are discarded by the
  // 0/1 factor rather than by a branch.
  volatile T* v = wave_vals;
  v[lid] = mine;
  for (int dist = 32; dist > 0; dist >>= 1) {
    const T other = v[(lid + dist) & 63];
    mine = mine + T(lid < dist) * other;
    v[lid] = mine;
  }
  if (lid == 0) partial[blockIdx.x] = mine;
}

// Work-items the device keeps resident for a kernel (the paper's global
// size), as a number of work-groups.
template <class K> int resident_groups(K kernel, int block, size_t lds, int cus) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return per_cu * cus;
}

template <class T, int F>
hipError_t launch_unrolled(const T* x, int64_t n, T* partial, int cap, int cus, int* groups, hipStream_t s) {
  static const int resident = resident_groups(design_unrolled_partials<T, F>, 64, 0, cus);  // queried once
  *groups = resident < cap ? resident : cap;
  hipLaunchKernelGGL((design_unrolled_partials<T, F>), dim3(*groups), dim3(64), 0, s, x, n, partial);
  return hipGetLastError();
}

template <class T>
hipError_t run(const T* x, int64_t n, int variant, int unroll, T* out, T* partial, int cap, int cus,
               hipStream_t s) {
  int groups = 0;
  hipError_t e;
  if (variant == 0) {
    constexpr int kBlock = 256;
    static const int resident = resident_groups(design_strided_partials<T>, kBlock, kBlock * sizeof(T), cus);
    groups = resident < cap ? resident : cap;
    hipLaunchKernelGGL((design_strided_partials<T>), dim3(groups), dim3(kBlock), kBlock * sizeof(T), s, x, n,
                       partial);
    e = hipGetLastError();
  } else {
    switch (unroll) {
      case 1: e = launch_unrolled<T, 1>(x, n, partial, cap, cus, &groups, s); break;
      case 2: e = launch_unrolled<T, 2>(x, n, partial, cap, cus, &groups, s); break;
      case 3: e = launch_unrolled<T, 3>(x, n, partial, cap, cus, &groups, s); break;
      case 4: e = launch_unrolled<T, 4>(x, n, partial, cap, cus, &groups, s); break;
      case 5: e = launch_unrolled<T, 5>(x, n, partial, cap, cus, &groups, s); break;
      case 6: e = launch_unrolled<T, 6>(x, n, partial, cap, cus, &groups, s); break;
      case 7: e = launch_unrolled<T, 7>(x, n, partial, cap, cus, &groups, s); break;
      case 8: e = launch_unrolled<T, 8>(x, n, partial, cap, cus, &groups, s); break;
      case 16: e = launch_unrolled<T, 16>(x, n, partial, cap, cus, &groups, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  constexpr int kFinalBlock = 1024;
  hipLaunchKernelGGL((design_final<T>), dim3(1), dim3(kFinalBlock), kFinalBlock * sizeof(T), s,
                     (const T*)partial, (int64_t)groups, out);
  return hipGetLastError();
}

}  // namespace

hipError_t paper_design_reduce(const void* x, int64_t n, rd_dtype dt, int variant, int unroll, void* out,
                               void* partial, int cap, int cus, hipStream_t s) {
  if (dt == RD_F32) return run<float>((const float*)x, n, variant, unroll, (float*)out, (float*)partial, cap, cus, s);
  // int32 sums wrap modulo 2^32: accumulate the same bits as unsigned
  if (dt == RD_I32) return run<uint32_t>((const uint32_t*)x, n, variant, unroll, (uint32_t*)out, (uint32_t*)partial, cap, cus, s);
  return hipErrorInvalidValue;
}

}  // namespace rd
