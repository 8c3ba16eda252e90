// rowreduce.hip -- row-wise reduction of a float32 matrix and its gradient.
//
// Forward: y[r] = x[r,0] (+) ... (+) x[r,cols-1] for (+) in {+, max, min, x},
// one persistent work-group per row at a time, the row walked in chunks of
// kChunk columns; each work-item owns 4 consecutive columns per stripe,
// loaded with one 16-byte load (four 4-byte loads when rows are not 16-byte
// aligned).
//   max/min also record the LOWEST column attaining the extreme: each lane
//     keeps an order-preserving integer key per accumulator slot plus the
//     chunk where it was first reached, and ties resolve to the smaller
//     column when lanes, wavefronts and slots are combined.
//   product also records, per row, the number of exact zeros, the first
//     zero's column and the product of the nonzero entries, and per chunk
//     the product of its nonzero entries (the state the gradient needs).
// Backward (grad = dy/dx * g):
//   sum     -> g[r] broadcast (write-only);
//   max/min -> g[r] at the saved column, 0 elsewhere (write-only);
//   product -> rows with >= 2 zeros: 0; one zero: g*prod(nonzeros) at the
//              zero; no zero: g * prod_{i<j} x * prod_{i>j} x, built from
//              chunk products and, inside a chunk, DPP prefix/suffix scans
//              over wavefronts and an LDS step over wavefronts -- no division.
#include "rd_device.hpp"
#include "rd_internal.hpp"

namespace rd {

namespace {

constexpr int kRowBlock = 256;             // work-items per group (4 wavefronts)
constexpr int kRowWaves = kRowBlock / 64;
constexpr int kPerLane = 64;               // elements per work-item per chunk
constexpr int64_t kChunk = (int64_t)kRowBlock * kPerLane;  // 16384 columns

struct ProdHeader {  // per-row product bookkeeping (16 bytes)
  int32_t zeros;
  int32_t first_zero;  // column of the first exact zero, -1 if none
  float pnz;           // product of the nonzero entries
  float reserved;
};

__host__ __device__ inline int64_t chunks_of(int64_t cols) { return (cols + kChunk - 1) / kChunk; }

// Order-preserving integer key of a float (-0 < +0); NaN maps to `nan_key`.
__device__ __forceinline__ int32_t float_key(float v, int32_t nan_key) {
  const int32_t b = __builtin_bit_cast(int32_t, v);
  const int32_t k = b ^ ((b >> 31) & 0x7FFFFFFF);
  return (v != v) ? nan_key : k;
}
__device__ __forceinline__ float key_float(int32_t k) {
  const int32_t b = k ^ ((k >> 31) & 0x7FFFFFFF);
  return __builtin_bit_cast(float, b);
}

// Load the 4 consecutive floats of stripe u at column `col` (missing columns
// of a ragged chunk take `fill`).  AL: the row pointer and cols keep every
// stripe 16-byte aligned, so one global_load_dwordx4 serves.
template <bool AL>
__device__ __forceinline__ void load_stripe(const float* __restrict__ row, int64_t col, int64_t cols,
                                            bool full, float fill, float (&v)[4]) {
  if (AL && (full || col + 3 < cols)) {
    const u32x4 q = __builtin_nontemporal_load((const u32x4*)(row + col));
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = lane_elem<float>(q, e);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (full || col + e < cols) ? row[col + e] : fill;
  }
}

template <bool AL>
__device__ __forceinline__ void store_stripe(float* __restrict__ row, int64_t col, int64_t cols,
                                             bool full, const float (&v)[4]) {
  if (AL && (full || col + 3 < cols)) {
    u32x4 q;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t b = __builtin_bit_cast(uint32_t, v[e]);
      q[e] = b;
    }
    __builtin_nontemporal_store(q, (u32x4*)(row + col));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (full || col + e < cols) row[col + e] = v[e];
  }
}

struct ProdAcc {  // chunk-level product state (16 bytes, combinable by DPP)
  double p;       // product of nonzero entries (float64: see the plain kernel's traits)
  int32_t zeros;
  int32_t first;  // smallest zero column, INT32_MAX if none
};

}  // namespace

// ------------------------------------------------------------------ forward

template <Op O, bool AL>
__global__ __launch_bounds__(kRowBlock) void row_fwd_kernel(const float* __restrict__ x, int64_t rows,
                                                            int64_t cols, float* __restrict__ y,
                                                            void* __restrict__ saved) {
  constexpr int U = kPerLane / 4;  // stripes of 4 consecutive columns per chunk
  const int t = threadIdx.x;
  const int64_t nch = chunks_of(cols);
  __shared__ float lds_f[kRowWaves];
  __shared__ uint64_t lds_u[kRowWaves];
  __shared__ ProdAcc lds_p[kRowWaves];

  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const float* __restrict__ row = x + r * cols;
    if constexpr (O == Op::Sum) {
      float acc[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[u][e] = 0.0f;
      for (int64_t k = 0; k < nch; ++k) {
        const int64_t c0 = k * kChunk;
        const bool full = c0 + kChunk <= cols;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float v[4];
          load_stripe<AL>(row, c0 + ((int64_t)u * kRowBlock + t) * 4, cols, full, 0.0f, v);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[u][e] += v[e];
        }
      }
      float mine = 0.0f;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) mine += acc[u][e];
      const float tot = block_reduce(mine, 0.0f, [](float a, float b) { return a + b; }, lds_f);
      if (t == 0) y[r] = tot;
      __syncthreads();
    } else if constexpr (O == Op::Max || O == Op::Min) {
      constexpr bool MAX = (O == Op::Max);
      constexpr int32_t NAN_KEY = MAX ? 0x7FFFFFFF : (int32_t)0x80000000;
      constexpr int32_t NONE_KEY = MAX ? (int32_t)0x80000000 : 0x7FFFFFFF;  // below/above every value
      int32_t best[U][4];
      int32_t at[U][4];  // chunk index where best was first reached
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          best[u][e] = NONE_KEY;
          at[u][e] = -1;
        }
      for (int64_t k = 0; k < nch; ++k) {
        const int64_t c0 = k * kChunk;
        const bool full = c0 + kChunk <= cols;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float v[4];
          const int64_t col = c0 + ((int64_t)u * kRowBlock + t) * 4;
          load_stripe<AL>(row, col, cols, full, 0.0f, v);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool valid = full || (col + e < cols);
            const int32_t key = float_key(v[e], NAN_KEY);
            const bool better = valid && (MAX ? key > best[u][e] : key < best[u][e]);
            best[u][e] = better ? key : best[u][e];
            at[u][e] = better ? (int32_t)k : at[u][e];
          }
        }
      }
      // Pack (key, column) so one unsigned max/min picks the extreme and, among
      // equal keys, the lowest column.
      uint64_t mine = MAX ? 0ull : ~0ull;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (at[u][e] < 0) continue;
          const uint32_t col = (uint32_t)((int64_t)at[u][e] * kChunk + ((int64_t)u * kRowBlock + t) * 4 + e);
          const uint32_t ukey = (uint32_t)best[u][e] ^ 0x80000000u;
          const uint64_t packed = MAX ? (((uint64_t)ukey << 32) | (uint64_t)(0xFFFFFFFFu - col))
                                      : (((uint64_t)ukey << 32) | (uint64_t)col);
          mine = MAX ? (packed > mine ? packed : mine) : (packed < mine ? packed : mine);
        }
      const uint64_t id = MAX ? 0ull : ~0ull;
      const uint64_t tot = block_reduce(
          mine, id, [](uint64_t a, uint64_t b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); }, lds_u);
      if (t == 0) {
        int64_t col = -1;
        float val = MAX ? -__builtin_inff() : __builtin_inff();
        if (tot != id) {
          const uint32_t lo = (uint32_t)tot;
          col = MAX ? (int64_t)(0xFFFFFFFFu - lo) : (int64_t)lo;
          const int32_t key = (int32_t)((uint32_t)(tot >> 32) ^ 0x80000000u);
          val = (key == NAN_KEY) ? __builtin_nanf("") : key_float(key);
        }
        y[r] = val;
        ((int64_t*)saved)[r] = col;
      }
      __syncthreads();
    } else {  // product
      ProdHeader* hdr = (ProdHeader*)saved;
      float* chunk_prod = (float*)((char*)saved + rows * (int64_t)sizeof(ProdHeader));
      int32_t zeros = 0, first = INT32_MAX;
      double pnz = 1.0;
      auto comb = [](ProdAcc a, ProdAcc b) {
        return ProdAcc{a.p * b.p, a.zeros + b.zeros, a.first < b.first ? a.first : b.first};
      };
      for (int64_t k = 0; k < nch; ++k) {
        const int64_t c0 = k * kChunk;
        const bool full = c0 + kChunk <= cols;
        double p = 1.0;
        int32_t z = 0, fz = INT32_MAX;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float v[4];
          const int64_t col = c0 + ((int64_t)u * kRowBlock + t) * 4;
          load_stripe<AL>(row, col, cols, full, 1.0f, v);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool zero = (v[e] == 0.0f);
            p = zero ? p : p * (double)v[e];
            z += zero ? 1 : 0;
            fz = (zero && fz == INT32_MAX) ? (int32_t)(col + e) : fz;
          }
        }
        const ProdAcc tot = block_reduce(ProdAcc{p, z, fz}, ProdAcc{1.0, 0, INT32_MAX}, comb, lds_p);
        if (t == 0) {
          chunk_prod[r * nch + k] = (float)tot.p;
          zeros += tot.zeros;
          first = tot.first < first ? tot.first : first;
          pnz *= tot.p;
        }
        __syncthreads();
      }
      if (t == 0) {
        hdr[r] = ProdHeader{zeros, first == INT32_MAX ? -1 : first, (float)pnz, 0.0f};
        y[r] = zeros > 0 ? 0.0f * (float)pnz : (float)pnz;
      }
    }
  }
}

// ------------------------------------------------------------------ backward

// sum / max / min / product rows with zeros: write-only fill.
template <Op O, bool AL>
__global__ __launch_bounds__(kRowBlock) void row_bwd_kernel(const float* __restrict__ x,
                                                            const float* __restrict__ g,
                                                            const void* __restrict__ saved,
                                                            int64_t rows, int64_t cols,
                                                            float* __restrict__ grad) {
  constexpr int U = kPerLane / 4;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t nch = chunks_of(cols);
  __shared__ float lds_tot[kRowWaves][U];

  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const float gr = g[r];
    float* __restrict__ out = grad + r * cols;
    int64_t hot = -1;  // the one column receiving a nonzero value (or -1: every column)
    float hot_val = 0.0f, fill = 0.0f;
    bool scan = false;
    if constexpr (O == Op::Sum) {
      fill = gr;
    } else if constexpr (O == Op::Max || O == Op::Min) {
      hot = ((const int64_t*)saved)[r];
      hot_val = gr;
    } else {
      const ProdHeader h = ((const ProdHeader*)saved)[r];
      if (h.zeros == 1) {
        hot = h.first_zero;
        hot_val = gr * h.pnz;
      } else if (h.zeros == 0) {
        scan = true;
      }
    }

    if (!scan) {
      for (int64_t k = 0; k < nch; ++k) {
        const int64_t c0 = k * kChunk;
        const bool full = c0 + kChunk <= cols;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t col = c0 + ((int64_t)u * kRowBlock + t) * 4;
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (col + e == hot) ? hot_val : fill;
          store_stripe<AL>(out, col, cols, full, v);
        }
      }
      continue;
    }

    // Product row without zeros: exclusive products, no division.
    const float* __restrict__ row = x + r * cols;
    const float* chunk_prod = (const float*)((const char*)saved + rows * (int64_t)sizeof(ProdHeader)) + r * nch;
    auto mul = [](float a, float b) { return a * b; };
    for (int64_t k = 0; k < nch; ++k) {
      const int64_t c0 = k * kChunk;
      const bool full = c0 + kChunk <= cols;
      float CP = 1.0f, CS = 1.0f;  // products of the chunks before / after this one
      for (int64_t j = 0; j < k; ++j) CP *= chunk_prod[j];
      for (int64_t j = k + 1; j < nch; ++j) CS *= chunk_prod[j];

      float v[U][4], m[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        load_stripe<AL>(row, c0 + ((int64_t)u * kRowBlock + t) * 4, cols, full, 1.0f, v[u]);
        float p = v[u][0];
#pragma unroll
        for (int e = 1; e < 4; ++e) p *= v[u][e];
        m[u] = p;  // product of this work-item's 4 columns of stripe u
      }
      // Across the 64 lanes: exclusive prefix (lanes below) and suffix (lanes above).
      float E[U], F[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float inc = wave_scan_incl(m[u], 1.0f, mul);
        E[u] = wave_shift_up(inc, 1.0f);
        const float rinc = wave_scan_incl(wave_reverse(m[u]), 1.0f, mul);
        F[u] = wave_reverse(wave_shift_up(rinc, 1.0f));
        if (lane == 63) lds_tot[wave][u] = inc;  // wavefront product of stripe u
      }
      __syncthreads();
      // Across wavefronts and stripes.
      float SP = 1.0f;  // product of whole stripes before u
      float R[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float before = 1.0f, after = 1.0f, all = 1.0f;
#pragma unroll
        for (int w2 = 0; w2 < kRowWaves; ++w2) {
          const float q = lds_tot[w2][u];
          if (w2 < wave) before *= q;
          if (w2 > wave) after *= q;
          all *= q;
        }
        E[u] *= before;
        F[u] *= after;
        R[u] = all;
      }
      float SS[U];  // product of whole stripes after u
      {
        float acc = 1.0f;
#pragma unroll
        for (int u = U - 1; u >= 0; --u) {
          SS[u] = acc;
          acc *= R[u];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float left = gr * CP * SP * E[u];
        const float right = F[u] * SS[u] * CS;
        SP *= R[u];
        float o[4];
        float pre = 1.0f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float suf = 1.0f;
#pragma unroll
          for (int e2 = e + 1; e2 < 4; ++e2) suf *= v[u][e2];
          o[e] = left * pre * suf * right;
          pre *= v[u][e];
        }
        store_stripe<AL>(out, c0 + ((int64_t)u * kRowBlock + t) * 4, cols, full, o);
      }
      __syncthreads();  // lds_tot is rewritten by the next chunk
    }
  }
}

// ------------------------------------------------------------------ host side

size_t rowreduce_saved_bytes(rd_op op, int64_t rows, int64_t cols) {
  switch (op) {
    case RD_SUM: return 0;
    case RD_MAX:
    case RD_MIN: return (size_t)rows * 8;
    case RD_PROD: return (size_t)rows * sizeof(ProdHeader) + (size_t)rows * chunks_of(cols) * 4;
    default: return 0;
  }
}

namespace {
// Persistent grid over rows: at most 8 work-groups per CU.
int row_grid(int64_t rows, int cus) {
  const int64_t g = (int64_t)cus * 8;
  return (int)(rows < g ? rows : g);
}

template <Op O, bool AL>
hipError_t fwd_launch(const float* x, int64_t rows, int64_t cols, float* y, void* saved, int cus,
                      hipStream_t s) {
  hipLaunchKernelGGL((row_fwd_kernel<O, AL>), dim3(row_grid(rows, cus)), dim3(kRowBlock), 0, s, x, rows,
                     cols, y, saved);
  return hipGetLastError();
}

template <Op O, bool AL>
hipError_t bwd_launch(const float* x, const float* g, const void* saved, int64_t rows, int64_t cols,
                      float* grad, int cus, hipStream_t s) {
  hipLaunchKernelGGL((row_bwd_kernel<O, AL>), dim3(row_grid(rows, cus)), dim3(kRowBlock), 0, s, x, g,
                     saved, rows, cols, grad);
  return hipGetLastError();
}
}  // namespace

hipError_t rowreduce_fwd(const float* x, int64_t rows, int64_t cols, rd_op op, float* y, void* saved,
                         int cus, hipStream_t s) {
  const bool v4 = (cols % 4 == 0) && ((uintptr_t)x % 16 == 0);
  switch (op) {
    case RD_SUM: return v4 ? fwd_launch<Op::Sum, true>(x, rows, cols, y, saved, cus, s) : fwd_launch<Op::Sum, false>(x, rows, cols, y, saved, cus, s);
    case RD_MAX: return v4 ? fwd_launch<Op::Max, true>(x, rows, cols, y, saved, cus, s) : fwd_launch<Op::Max, false>(x, rows, cols, y, saved, cus, s);
    case RD_MIN: return v4 ? fwd_launch<Op::Min, true>(x, rows, cols, y, saved, cus, s) : fwd_launch<Op::Min, false>(x, rows, cols, y, saved, cus, s);
    case RD_PROD: return v4 ? fwd_launch<Op::Prod, true>(x, rows, cols, y, saved, cus, s) : fwd_launch<Op::Prod, false>(x, rows, cols, y, saved, cus, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t rowreduce_bwd(const float* x, const float* g, const void* saved, int64_t rows, int64_t cols,
                         rd_op op, float* grad, int cus, hipStream_t s) {
  const bool v4 = (cols % 4 == 0) && ((uintptr_t)grad % 16 == 0) && (op != RD_PROD || (uintptr_t)x % 16 == 0);
  switch (op) {
    case RD_SUM: return v4 ? bwd_launch<Op::Sum, true>(x, g, saved, rows, cols, grad, cus, s) : bwd_launch<Op::Sum, false>(x, g, saved, rows, cols, grad, cus, s);
    case RD_MAX: return v4 ? bwd_launch<Op::Max, true>(x, g, saved, rows, cols, grad, cus, s) : bwd_launch<Op::Max, false>(x, g, saved, rows, cols, grad, cus, s);
    case RD_MIN: return v4 ? bwd_launch<Op::Min, true>(x, g, saved, rows, cols, grad, cus, s) : bwd_launch<Op::Min, false>(x, g, saved, rows, cols, grad, cus, s);
    case RD_PROD: return v4 ? bwd_launch<Op::Prod, true>(x, g, saved, rows, cols, grad, cus, s) : bwd_launch<Op::Prod, false>(x, g, saved, rows, cols, grad, cus, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rd
