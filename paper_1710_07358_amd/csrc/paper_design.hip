// paper_design.hip -- the paper's own kernel designs on gfx950, kept as
// measured baselines for the tuned kernels (sum of int32 or float32 only).
//
// variant 0: the two-stage reduction of Section 2.3 (its stage-1 listing):
//   GS work-items (the most the device keeps resident) each accumulate
//   x[gid], x[gid + GS], ... with one scalar load per step, write a local
//   scratch array, reduce it with a halving tree and a barrier per level,
//   and work-item 0 writes one partial per work-group; a second launch
//   reduces the partials the same way in one work-group.
// variant 1: the new approach of Section 3: the global loop unrolled F times
//   (work-item reads F consecutive elements, stride GS*F) with the algebraic
//   guard -- an out-of-range term contributes (0) * x[0], as the text
//   describes, so nothing is read past the end -- and the barrier-free
//   algebraic tree of the "Avoiding Divergences" listing.  That tree is only
//   correct when the work-group is one wavefront, so variant 1 runs 64
//   work-items per group.  Stage 2 as in variant 0.
#include "rd_device.hpp"
#include "rd_internal.hpp"

namespace rd {

namespace {

template <class T>
__global__ __launch_bounds__(1024) void two_stage_stage1(const T* __restrict__ x, int64_t n, T* __restrict__ partial) {
  extern __shared__ unsigned char smem[];
  T* scratch = (T*)smem;
  const int64_t gs = (int64_t)gridDim.x * blockDim.x;
  T acc = T(0);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) acc += x[i];
  const int lid = threadIdx.x;
  scratch[lid] = acc;
  __syncthreads();
  for (int offset = blockDim.x / 2; offset > 0; offset >>= 1) {
    if (lid < offset) scratch[lid] += scratch[lid + offset];
    __syncthreads();
  }
  if (lid == 0) partial[blockIdx.x] = scratch[0];
}

template <class T>
__global__ __launch_bounds__(1024) void two_stage_stage2(const T* __restrict__ partial, int64_t count,
                                                         T* __restrict__ out) {
  extern __shared__ unsigned char smem[];
  T* scratch = (T*)smem;
  const int lid = threadIdx.x;
  T acc = T(0);
  for (int64_t i = lid; i < count; i += blockDim.x) acc += partial[i];
  scratch[lid] = acc;
  __syncthreads();
  for (int offset = blockDim.x / 2; offset > 0; offset >>= 1) {
    if (lid < offset) scratch[lid] += scratch[lid + offset];
    __syncthreads();
  }
  if (lid == 0) *out = scratch[0];
}

template <class T, int F>
__global__ __launch_bounds__(64) void unrolled_stage1(const T* __restrict__ x, int64_t n, T* __restrict__ partial) {
  __shared__ T scratch_mem[64];
  volatile T* scratch = scratch_mem;  // every step goes through LDS, as in the listing
  const int64_t gs = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  T acc = T(0);
  for (int64_t pos = gid * F; pos < n; pos += gs * F) {
    T step = T(0);
#pragma unroll
    for (int k = 0; k < F; ++k) {
      const int64_t i = pos + k;
      const bool in = i < n;
      step += (T)in * x[in ? i : 0];  // (i < n) * x[i], reading x[0] when out of range
    }
    acc += step;
  }
  const int lid = threadIdx.x;
  scratch[lid] = acc;
  for (int p = 32; p > 0; p >>= 1) {  // barrier-free: one wavefront moves in lockstep
    const int flag = lid < p;
    scratch[lid] += (T)flag * scratch[lid + flag * p];
  }
  if (lid == 0) partial[blockIdx.x] = scratch[0];
}

// Work-items the device keeps resident for a kernel (the paper's GS), as a
// number of work-groups.
template <class K> int resident_groups(K kernel, int block, size_t lds, int cus) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return per_cu * cus;
}

template <class T, int F>
hipError_t launch_unrolled(const T* x, int64_t n, T* partial, int cap, int cus, int* groups, hipStream_t s) {
  static const int resident = resident_groups(unrolled_stage1<T, F>, 64, 0, cus);  // queried once
  int g = resident;
  g = g > cap ? cap : g;
  hipLaunchKernelGGL((unrolled_stage1<T, F>), dim3(g), dim3(64), 0, s, x, n, partial);
  *groups = g;
  return hipGetLastError();
}

template <class T>
hipError_t run(const T* x, int64_t n, int variant, int unroll, T* out, T* partial, int cap, int cus,
               hipStream_t s) {
  int groups = 0;
  hipError_t e;
  if (variant == 0) {
    const int block = 256;
    static const int resident = resident_groups(two_stage_stage1<T>, block, block * sizeof(T), cus);
    groups = resident;
    groups = groups > cap ? cap : groups;
    hipLaunchKernelGGL((two_stage_stage1<T>), dim3(groups), dim3(block), block * sizeof(T), s, x, n, partial);
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
  const int block2 = 1024;
  hipLaunchKernelGGL((two_stage_stage2<T>), dim3(1), dim3(block2), block2 * sizeof(T), s, (const T*)partial,
                     (int64_t)groups, out);
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
