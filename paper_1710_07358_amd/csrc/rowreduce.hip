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

#include <algorithm>

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
// stripe 16-byte aligned, so one global_load_dwordx4 serves.  NT: non-temporal.
template <bool AL, bool NT = true>
__device__ __forceinline__ void load_stripe(const float* __restrict__ row, int64_t col, int64_t cols,
                                            bool full, float fill, float (&v)[4]) {
  if (AL && (full || col + 3 < cols)) {
    const u32x4 q = load16<NT>((const u32x4*)(row + col));
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = lane_elem<float>(q, e);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (full || col + e < cols) ? row[col + e] : fill;
  }
}

template <bool AL, bool NT = true>
__device__ __forceinline__ void store_stripe(float* __restrict__ row, int64_t col, int64_t cols,
                                             bool full, const float (&v)[4]) {
  if (AL && (full || col + 3 < cols)) {
    u32x4 q;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t b = __builtin_bit_cast(uint32_t, v[e]);
      q[e] = b;
    }
    if constexpr (NT) __builtin_nontemporal_store(q, (u32x4*)(row + col));
    else *(u32x4*)(row + col) = q;
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

// Each step covers S stripes of 4 consecutive columns per work-item:
// kRowBlock * 4 * S columns.  S divides kPerLane / 4, so product chunks are
// whole numbers of steps.
template <int S> constexpr int64_t row_step() { return (int64_t)kRowBlock * 4 * S; }

// Walk columns [cb, ce) of a row in steps (cb a multiple of the step; ce a
// multiple of it or the row's end): body(v, c0, full) folds the step at c0.
// Whole steps are software-pipelined -- the next step's loads are issued
// before the current one is folded -- and use unguarded loads; only a ragged
// last step takes the guarded path, filling missing columns with `fill`.
template <bool AL, bool NT, int S, class Body>
__device__ __forceinline__ void walk_steps(const float* __restrict__ row, int64_t cb, int64_t ce, int64_t cols,
                                           float fill, int t, Body body) {
  constexpr int64_t STEP = row_step<S>();
  int64_t c0 = cb;
  if (c0 + STEP <= ce) {
    float cur[S][4], nxt[S][4];
#pragma unroll
    for (int u = 0; u < S; ++u) load_stripe<AL, NT>(row, c0 + ((int64_t)u * kRowBlock + t) * 4, cols, true, fill, cur[u]);
    for (; c0 + STEP <= ce; c0 += STEP) {
      const bool more = c0 + 2 * STEP <= ce;
      if (more) {
#pragma unroll
        for (int u = 0; u < S; ++u)
          load_stripe<AL, NT>(row, c0 + STEP + ((int64_t)u * kRowBlock + t) * 4, cols, true, fill, nxt[u]);
      }
      body(cur, c0, true);
      if (more) {
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) cur[u][e] = nxt[u][e];
      }
    }
  }
  if (c0 < ce) {
    float v[S][4];
#pragma unroll
    for (int u = 0; u < S; ++u) load_stripe<AL, NT>(row, c0 + ((int64_t)u * kRowBlock + t) * 4, cols, false, fill, v[u]);
    body(v, c0, false);
  }
}

template <Op O, bool AL, int S, bool NT>
__global__ __launch_bounds__(kRowBlock) void row_fwd_kernel(const float* __restrict__ x, int64_t rows,
                                                            int64_t cols, float* __restrict__ y,
                                                            void* __restrict__ saved) {
  constexpr int64_t STEP = row_step<S>();
  static_assert(kChunk % STEP == 0, "a chunk is a whole number of steps");
  const int t = threadIdx.x;
  __shared__ float lds_f[kRowWaves];
  __shared__ uint64_t lds_u[kRowWaves];
  __shared__ ProdAcc lds_p[kRowWaves];

  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const float* __restrict__ row = x + r * cols;
    if constexpr (O == Op::Sum) {
      float acc[S][4];
#pragma unroll
      for (int u = 0; u < S; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[u][e] = 0.0f;
      walk_steps<AL, NT, S>(row, 0, cols, cols, 0.0f, t, [&](const float (&v)[S][4], int64_t, bool) {
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[u][e] += v[u][e];
      });
      float mine = 0.0f;
#pragma unroll
      for (int u = 0; u < S; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) mine += acc[u][e];
      const float tot = block_reduce(mine, 0.0f, [](float a, float b) { return a + b; }, lds_f);
      if (t == 0) y[r] = tot;
      __syncthreads();
    } else if constexpr (O == Op::Max || O == Op::Min) {
      constexpr bool MAX = (O == Op::Max);
      constexpr int32_t NAN_KEY = MAX ? 0x7FFFFFFF : (int32_t)0x80000000;
      const float ident = MAX ? -__builtin_inff() : __builtin_inff();
      // Per slot: the IEEE 754-2019 maximum (minimum) so far and the step at
      // which its bits last changed.  Equal values leave the bits alone, so the
      // first occurrence is kept; once a NaN is in, the slot stops updating.
      float best[S][4];
      int32_t at[S][4];
      walk_steps<AL, NT, S>(row, 0, cols, cols, ident, t, [&](const float (&v)[S][4], int64_t c0, bool full) {
        const int64_t st = c0 / STEP;
        if (st == 0) {
#pragma unroll
          for (int u = 0; u < S; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const bool valid = full || (((int64_t)u * kRowBlock + t) * 4 + e < cols);
              best[u][e] = v[u][e];
              at[u][e] = valid ? 0 : -1;
            }
        } else {
#pragma unroll
          for (int u = 0; u < S; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float nb = MAX ? __builtin_elementwise_maximum(best[u][e], v[u][e])
                                   : __builtin_elementwise_minimum(best[u][e], v[u][e]);
              const bool changed = (__builtin_bit_cast(uint32_t, nb) != __builtin_bit_cast(uint32_t, best[u][e])) &&
                                   (best[u][e] == best[u][e]);
              at[u][e] = changed ? (int32_t)st : at[u][e];
              best[u][e] = nb;
            }
        }
      });
      // Pack (key, column) so one unsigned max/min picks the extreme and, among
      // equal keys, the lowest column.
      uint64_t mine = MAX ? 0ull : ~0ull;
#pragma unroll
      for (int u = 0; u < S; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (at[u][e] < 0) continue;
          const uint32_t col = (uint32_t)((int64_t)at[u][e] * STEP + ((int64_t)u * kRowBlock + t) * 4 + e);
          const uint32_t ukey = (uint32_t)float_key(best[u][e], NAN_KEY) ^ 0x80000000u;
          const uint64_t packed = MAX ? (((uint64_t)ukey << 32) | (uint64_t)(0xFFFFFFFFu - col))
                                      : (((uint64_t)ukey << 32) | (uint64_t)col);
          mine = MAX ? (packed > mine ? packed : mine) : (packed < mine ? packed : mine);
        }
      const uint64_t id = MAX ? 0ull : ~0ull;
      const uint64_t tot = block_reduce(
          mine, id, [](uint64_t a, uint64_t b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); }, lds_u);
      if (t == 0) {
        int64_t col = -1;
        float val = ident;
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
      const int64_t nch = chunks_of(cols);
      ProdHeader* hdr = (ProdHeader*)saved;
      float* chunk_prod = (float*)((char*)saved + rows * (int64_t)sizeof(ProdHeader));
      int32_t zeros = 0, first = INT32_MAX;
      double pnz = 1.0;
      auto comb = [](ProdAcc a, ProdAcc b) {
        return ProdAcc{a.p * b.p, a.zeros + b.zeros, a.first < b.first ? a.first : b.first};
      };
      for (int64_t k = 0; k < nch; ++k) {
        double p = 1.0;
        int32_t z = 0, fz = INT32_MAX;
        const int64_t ce = (k + 1) * kChunk < cols ? (k + 1) * kChunk : cols;
        walk_steps<AL, NT, S>(row, k * kChunk, ce, cols, 1.0f, t, [&](const float (&v)[S][4], int64_t c0, bool) {
          // A zero multiplies as 1.0 (exactly p), so the product needs no
          // 64-bit select; zeros are counted, and the first located, only in
          // the steps where some lane of the wavefront holds one.
          bool anyz = false;
#pragma unroll
          for (int u = 0; u < S; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const bool zero = (v[u][e] == 0.0f);
              anyz = anyz || zero;
              p *= (double)(zero ? 1.0f : v[u][e]);
            }
          if (__builtin_amdgcn_ballot_w64(anyz) != 0ull) {
#pragma unroll
            for (int u = 0; u < S; ++u)
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const bool zero = (v[u][e] == 0.0f);
                z += zero ? 1 : 0;
                const int32_t col = (int32_t)(c0 + ((int64_t)u * kRowBlock + t) * 4 + e);
                fz = (zero && col < fz) ? col : fz;
              }
          }
        });
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

// Exclusive products of one zero-free row, chunk by chunk (see the file header).
template <bool AL>
__device__ __forceinline__ void prod_scan_row(const float* __restrict__ row, const float* __restrict__ chunk_prod,
                              int64_t cols, float gr, float* __restrict__ out,
                              float (&lds_tot)[kRowWaves][kPerLane / 4]) {
  constexpr int U = kPerLane / 4;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t nch = chunks_of(cols);
  auto mul = [](float a, float b) { return a * b; };
  float CP = 1.0f;  // product of the chunks before this one (running)
  for (int64_t k = 0; k < nch; ++k) {
    const int64_t c0 = k * kChunk;
    const bool full = c0 + kChunk <= cols;
    // product of the chunks after this one: one load per lane, then the wavefront
    float CS = 1.0f;
    for (int64_t j = k + 1 + lane; j < nch; j += 64) CS *= chunk_prod[j];
    CS = wave_reduce(CS, 1.0f, mul);

    float v[U][4], m[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      load_stripe<AL>(row, c0 + ((int64_t)u * kRowBlock + t) * 4, cols, full, 1.0f, v[u]);
      m[u] = (v[u][0] * v[u][1]) * (v[u][2] * v[u][3]);  // product of this work-item's 4 columns
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
    float SP = 1.0f;  // product of whole stripes before u
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float left = gr * CP * SP * E[u];
      const float right = F[u] * SS[u] * CS;
      SP *= R[u];
      const float p01 = v[u][0] * v[u][1], p23 = v[u][2] * v[u][3];
      float o[4];
      o[0] = left * (v[u][1] * p23) * right;
      o[1] = left * (v[u][0] * p23) * right;
      o[2] = left * (p01 * v[u][3]) * right;
      o[3] = left * (p01 * v[u][2]) * right;
      store_stripe<AL>(out, c0 + ((int64_t)u * kRowBlock + t) * 4, cols, full, o);
    }
    CP *= chunk_prod[k];
    __syncthreads();  // lds_tot is rewritten by the next chunk
  }
}

// Product rows without zeros: grad = g * (prefix product) * (suffix
// product), per row, persistent over rows.  Rows with zeros are written by
// the write-only kernel below.
template <bool AL, int S, bool NT>
__global__ __launch_bounds__(kRowBlock) void row_bwd_kernel(const float* __restrict__ x,
                                                            const float* __restrict__ g,
                                                            const void* __restrict__ saved,
                                                            int64_t rows, int64_t cols,
                                                            float* __restrict__ grad) {
  __shared__ float lds_tot[kRowWaves][kPerLane / 4];
  const int64_t nch = chunks_of(cols);
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const ProdHeader h = ((const ProdHeader*)saved)[r];
    if (h.zeros != 0) continue;
    const float* cp = (const float*)((const char*)saved + rows * (int64_t)sizeof(ProdHeader)) + r * nch;
    prod_scan_row<AL>(x + r * cols, cp, cols, g[r], grad + r * cols, lds_tot);
  }
}

// Write-only gradients (sum; min/max; product rows with zeros), one tile of
// kRowBlock x 4 columns per work-group and one 16-byte store per work-item,
// over a flat grid of rows x tiles: for pure writes, many short work-groups
// keep more stores in flight than a persistent loop (measured on MI355X:
// 6.9 TB/s against 6.2 TB/s).  Product rows without zeros are skipped here;
// the persistent kernel above scans them.
template <Op O, bool AL, bool NT>
__global__ __launch_bounds__(kRowBlock) void row_fill_kernel(const float* __restrict__ g,
                                                             const void* __restrict__ saved, int64_t rows,
                                                             int64_t cols, int64_t tiles, double inv_tiles,
                                                             float* __restrict__ grad) {
  const int64_t total = rows * tiles;
  for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {  // one pass unless the grid was capped
    int64_t r = (int64_t)((double)b * inv_tiles);  // b / tiles, then corrected
    if (r * tiles > b) --r;
    if ((r + 1) * tiles <= b) ++r;
    const int64_t col = (b - r * tiles) * (kRowBlock * 4) + (int64_t)threadIdx.x * 4;
    if (col >= cols) continue;
    const float gr = g[r];
    int64_t hot = -1;
    float hot_val = 0.0f, fill = 0.0f;
    if constexpr (O == Op::Sum) {
      fill = gr;
    } else if constexpr (O == Op::Max || O == Op::Min) {
      hot = ((const int64_t*)saved)[r];
      hot_val = gr;
    } else {
      const ProdHeader h = ((const ProdHeader*)saved)[r];
      if (h.zeros == 0) continue;
      if (h.zeros == 1) {
        hot = h.first_zero;
        hot_val = gr * h.pnz;
      }
    }
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (col + e == hot) ? hot_val : fill;
    store_stripe<AL, NT>(grad + r * cols, col, cols, col + 4 <= cols, v);
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
// Persistent grid over rows: blocks_per_cu work-groups per CU.
int row_grid(int64_t rows, int cus, int bpc) {
  const int64_t g = (int64_t)cus * bpc;
  return (int)(rows < g ? rows : g);
}

template <Op O, bool AL, int S>
hipError_t fwd_launch(const float* x, int64_t rows, int64_t cols, float* y, void* saved, int grid, bool nt,
                      hipStream_t s) {
  if (nt) hipLaunchKernelGGL((row_fwd_kernel<O, AL, S, true>), dim3(grid), dim3(kRowBlock), 0, s, x, rows, cols, y, saved);
  else hipLaunchKernelGGL((row_fwd_kernel<O, AL, S, false>), dim3(grid), dim3(kRowBlock), 0, s, x, rows, cols, y, saved);
  return hipGetLastError();
}

template <bool AL, int S>
hipError_t bwd_launch(const float* x, const float* g, const void* saved, int64_t rows, int64_t cols, float* grad,
                      int grid, bool nt, hipStream_t s) {
  if (nt) hipLaunchKernelGGL((row_bwd_kernel<AL, S, true>), dim3(grid), dim3(kRowBlock), 0, s, x, g, saved, rows, cols, grad);
  else hipLaunchKernelGGL((row_bwd_kernel<AL, S, false>), dim3(grid), dim3(kRowBlock), 0, s, x, g, saved, rows, cols, grad);
  return hipGetLastError();
}

template <Op O, bool AL>
hipError_t fwd_s(int S, const float* x, int64_t rows, int64_t cols, float* y, void* saved, int grid, bool nt,
                 hipStream_t s) {
  switch (S) {
    case 1: return fwd_launch<O, AL, 1>(x, rows, cols, y, saved, grid, nt, s);
    case 2: return fwd_launch<O, AL, 2>(x, rows, cols, y, saved, grid, nt, s);
    case 4: return fwd_launch<O, AL, 4>(x, rows, cols, y, saved, grid, nt, s);
    case 8: return fwd_launch<O, AL, 8>(x, rows, cols, y, saved, grid, nt, s);
  }
  return hipErrorInvalidValue;
}

template <bool AL>
hipError_t bwd_s(int S, const float* x, const float* g, const void* saved, int64_t rows, int64_t cols, float* grad,
                 int grid, bool nt, hipStream_t s) {
  switch (S) {
    case 1: return bwd_launch<AL, 1>(x, g, saved, rows, cols, grad, grid, nt, s);
    case 2: return bwd_launch<AL, 2>(x, g, saved, rows, cols, grad, grid, nt, s);
    case 4: return bwd_launch<AL, 4>(x, g, saved, rows, cols, grad, grid, nt, s);
    case 8: return bwd_launch<AL, 8>(x, g, saved, rows, cols, grad, grid, nt, s);
  }
  return hipErrorInvalidValue;
}

template <Op O>
hipError_t fwd_op(bool al, int S, const float* x, int64_t rows, int64_t cols, float* y, void* saved, int grid,
                  bool nt, hipStream_t s) {
  return al ? fwd_s<O, true>(S, x, rows, cols, y, saved, grid, nt, s)
            : fwd_s<O, false>(S, x, rows, cols, y, saved, grid, nt, s);
}

template <Op O, bool AL>
hipError_t fill_launch(const float* g, const void* saved, int64_t rows, int64_t cols, float* grad, bool nt,
                       hipStream_t s) {
  const int64_t tiles = (cols + kRowBlock * 4 - 1) / (kRowBlock * 4);
  const int64_t blocks = std::min<int64_t>(rows * tiles, (int64_t)1 << 30);
  const double inv = 1.0 / (double)tiles;
  if (nt) hipLaunchKernelGGL((row_fill_kernel<O, AL, true>), dim3((unsigned)blocks), dim3(kRowBlock), 0, s, g, saved,
                             rows, cols, tiles, inv, grad);
  else hipLaunchKernelGGL((row_fill_kernel<O, AL, false>), dim3((unsigned)blocks), dim3(kRowBlock), 0, s, g, saved,
                          rows, cols, tiles, inv, grad);
  return hipGetLastError();
}

template <Op O>
hipError_t bwd_op(bool al, int S, const float* x, const float* g, const void* saved, int64_t rows, int64_t cols,
                  float* grad, int grid, bool nt, hipStream_t s) {
  hipError_t e = al ? fill_launch<O, true>(g, saved, rows, cols, grad, nt, s)
                    : fill_launch<O, false>(g, saved, rows, cols, grad, nt, s);
  if constexpr (O != Op::Prod) {
    return e;
  } else {
    if (e != hipSuccess) return e;
    // product rows without zeros need their row scanned
    return al ? bwd_s<true>(S, x, g, saved, rows, cols, grad, grid, nt, s)
              : bwd_s<false>(S, x, g, saved, rows, cols, grad, grid, nt, s);
  }
}
}  // namespace

hipError_t rowreduce_fwd(const float* x, int64_t rows, int64_t cols, rd_op op, float* y, void* saved, int cus,
                         const Launch& l, hipStream_t s) {
  const bool al = (cols % 4 == 0) && ((uintptr_t)x % 16 == 0);
  const int grid = row_grid(rows, cus, l.grid);
  switch (op) {
    case RD_SUM: return fwd_op<Op::Sum>(al, l.unroll, x, rows, cols, y, saved, grid, l.nontemporal, s);
    case RD_MAX: return fwd_op<Op::Max>(al, l.unroll, x, rows, cols, y, saved, grid, l.nontemporal, s);
    case RD_MIN: return fwd_op<Op::Min>(al, l.unroll, x, rows, cols, y, saved, grid, l.nontemporal, s);
    case RD_PROD: return fwd_op<Op::Prod>(al, l.unroll, x, rows, cols, y, saved, grid, l.nontemporal, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t rowreduce_bwd(const float* x, const float* g, const void* saved, int64_t rows, int64_t cols, rd_op op,
                         float* grad, int cus, const Launch& l, hipStream_t s) {
  const bool al = (cols % 4 == 0) && ((uintptr_t)grad % 16 == 0) && (op != RD_PROD || (uintptr_t)x % 16 == 0);
  const int grid = row_grid(rows, cus, l.grid);
  switch (op) {
    case RD_SUM: return bwd_op<Op::Sum>(al, l.unroll, x, g, saved, rows, cols, grad, grid, l.nontemporal, s);
    case RD_MAX: return bwd_op<Op::Max>(al, l.unroll, x, g, saved, rows, cols, grad, grid, l.nontemporal, s);
    case RD_MIN: return bwd_op<Op::Min>(al, l.unroll, x, g, saved, rows, cols, grad, grid, l.nontemporal, s);
    case RD_PROD: return bwd_op<Op::Prod>(al, l.unroll, x, g, saved, rows, cols, grad, grid, l.nontemporal, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rd
