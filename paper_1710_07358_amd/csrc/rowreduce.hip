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
//     zero's column, the product of the nonzero entries and where its
//     infinite or NaN entries are (none, one column, several), and per chunk
//     of kChunk columns the products of all chunks before it and of all
//     chunks after it, in float64 (the state the gradient needs).
// Backward (grad = dy/dx * g):
//   sum     -> g[r] broadcast (write-only);
//   max/min -> g[r] at the saved column, 0 elsewhere (write-only);
//   product -> rows with >= 2 zeros: 0; one zero: g*prod(nonzeros) at the
//              zero, 0 elsewhere (IEEE NaN where the other entries pair a
//              zero with an infinity or NaN) -- the store-only fill shape;
//              no zero: g * prod_{i<j} x * prod_{i>j} x, a persistent launch
//              over (row, chunk) tiles: the chunk's own exclusive prefix and
//              suffix products come from DPP scans over the lanes and over
//              the chunk's 64 wavefront pieces, the rest of the row from the
//              saved chunk prefix/suffix -- no division.
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
  int32_t nonfinite;   // infinite or NaN entries: -1 none, -2 two or more, else the only one's column
};

__host__ __device__ inline int64_t chunks_of(int64_t cols) { return (cols + kChunk - 1) / kChunk; }

// Product saved state: [ProdHeader x rows][prefix: double x rows x nch]
// [suffix: double x rows x nch]; prefix[r][k] is the product of the chunks
// of row r before chunk k, suffix[r][k] of the chunks after it.
__host__ __device__ inline double* prod_prefix(void* saved, int64_t rows) {
  return (double*)((char*)saved + rows * (int64_t)sizeof(ProdHeader));
}
__host__ __device__ inline double* prod_suffix(void* saved, int64_t rows, int64_t nch) {
  return prod_prefix(saved, rows) + rows * nch;
}

// Value of lane 63 - lane for 4- or 8-byte values (ds_bpermute per 32 bits).
template <class A> __device__ __forceinline__ A wave_flip(A v) {
  const int addr = (63 - (int)(threadIdx.x & 63)) << 2;
  if constexpr (sizeof(A) == 4) {
    return __builtin_bit_cast(A, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
  } else {
    static_assert(sizeof(A) == 8, "4- or 8-byte values");
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(A, (uint64_t)lo | ((uint64_t)hi << 32));
  }
}

// Exclusive prefix (lanes below) and suffix (lanes above) products over the
// 64 lanes of a wavefront; *total gets the product of all 64.
template <class A>
__device__ __forceinline__ void wave_excl_products(A v, A* before, A* after, A* total) {
  const auto mul = [](A a, A b) { return a * b; };
  const A inc = wave_scan_incl(v, A(1), mul);
  *before = wave_shift_up(inc, A(1));
  *total = readlane(inc, 63);
  const A rinc = wave_scan_incl(wave_flip(v), A(1), mul);
  *after = wave_flip(wave_shift_up(rinc, A(1)));
}

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
  double p;        // product of nonzero entries (float64: see the plain kernel's traits)
  uint32_t zeros;  // bits 0..30: count of exact zeros; bit 31: xor of their sign bits
                   // (a -0 counts 0x80000001, a +0 counts 1: 32-bit addition sums the
                   // counts, below 2^31 since cols < 2^31, and xors the signs)
  int32_t first;   // smallest zero column, INT32_MAX if none
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
// The prefetch inside the loop is unconditional (the last whole step is
// peeled), so the compiler's wait before the fold covers the current step's
// loads only, not the ones just issued.
template <bool AL, bool NT, int S, class Body>
__device__ __forceinline__ void walk_steps(const float* __restrict__ row, int64_t cb, int64_t ce, int64_t cols,
                                           float fill, int t, Body body) {
  constexpr int64_t STEP = row_step<S>();
  int64_t c0 = cb;
  if (c0 + STEP <= ce) {
    float cur[S][4];
#pragma unroll
    for (int u = 0; u < S; ++u) load_stripe<AL, NT>(row, c0 + ((int64_t)u * kRowBlock + t) * 4, cols, true, fill, cur[u]);
    for (; c0 + 2 * STEP <= ce; c0 += STEP) {
      float nxt[S][4];
#pragma unroll
      for (int u = 0; u < S; ++u)
        load_stripe<AL, NT>(row, c0 + STEP + ((int64_t)u * kRowBlock + t) * 4, cols, true, fill, nxt[u]);
      body(cur, c0, true);
#pragma unroll
      for (int u = 0; u < S; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) cur[u][e] = nxt[u][e];
    }
    body(cur, c0, true);
    c0 += STEP;
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
  // Product rows: count of infinite or NaN entries and the first one's
  // column, one pair per row parity.  Work-item 0 reads and re-arms a row's
  // pair after the row's last barrier; the other wavefronts may already be on
  // the next row, which uses the other pair, and cannot reach the row after it
  // before passing a barrier of the next row, which work-item 0 reaches only
  // after the re-arm.
  __shared__ unsigned lds_nf[2];
  __shared__ int32_t lds_nf_col[2];
  if constexpr (O == Op::Prod) {
    if (t < 2) {
      lds_nf[t] = 0u;
      lds_nf_col[t] = INT32_MAX;
    }
    __syncthreads();
  }
  int parity = 0;

  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x, parity ^= 1) {
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
#pragma unroll
      for (int u = 0; u < S; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {  // an empty row keeps these: y = ident, column -1
          best[u][e] = ident;
          at[u][e] = -1;
        }
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
      double* __restrict__ pre = prod_prefix(saved, rows) + r * nch;
      double* __restrict__ suf = prod_suffix(saved, rows, nch) + r * nch;
      uint32_t zeros = 0;
      int32_t first = INT32_MAX;
      double pnz = 1.0;  // running product of the chunks so far
      auto comb = [](ProdAcc a, ProdAcc b) {
        return ProdAcc{a.p * b.p, a.zeros + b.zeros, a.first < b.first ? a.first : b.first};
      };
      for (int64_t k = 0; k < nch; ++k) {
        double p = 1.0;
        uint32_t z = 0;
        int32_t fz = INT32_MAX;
        const int64_t ce = (k + 1) * kChunk < cols ? (k + 1) * kChunk : cols;
        walk_steps<AL, NT, S>(row, k * kChunk, ce, cols, 1.0f, t, [&](const float (&v)[S][4], int64_t c0, bool) {
          // Fast path: multiply the step in, unguarded.  A zero factor always
          // leaves +-0 or NaN, so while every lane's product stays a normal
          // number the step held no zero and q is exactly what the zero-aware
          // walk below would give.  Otherwise (a zero, or an infinity, NaN,
          // overflow or underflow in some lane) the wavefront redoes the step
          // from p: zeros multiply as 1.0 and are counted, the first located.
          double q = p;
#pragma unroll
          for (int u = 0; u < S; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) q *= (double)v[u][e];
          if (__builtin_amdgcn_ballot_w64(!__builtin_isnormal(q)) == 0ull) {
            p = q;
            return;
          }
#pragma unroll
          for (int u = 0; u < S; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const bool zero = (v[u][e] == 0.0f);
              p *= (double)(zero ? 1.0f : v[u][e]);
              z += zero ? (__builtin_bit_cast(uint32_t, v[u][e]) | 1u) : 0u;  // sign bit + 1
              const int32_t col = (int32_t)(c0 + ((int64_t)u * kRowBlock + t) * 4 + e);
              fz = (zero && col < fz) ? col : fz;
              if (!__builtin_isfinite(v[u][e])) {  // filled columns of a ragged step hold 1.0
                atomicAdd(&lds_nf[parity], 1u);
                atomicMin(&lds_nf_col[parity], col);
              }
            }
        });
        const ProdAcc tot = block_reduce(ProdAcc{p, z, fz}, ProdAcc{1.0, 0u, INT32_MAX}, comb, lds_p);
        if (t == 0) {
          pre[k] = pnz;     // chunks before k
          suf[k] = tot.p;   // this chunk; turned into the chunks after k below
          zeros += tot.zeros;
          first = tot.first < first ? tot.first : first;
          pnz *= tot.p;
        }
        __syncthreads();  // also makes suf[] visible to wavefront 0
      }
      // Products of the chunks after each chunk: wavefront 0 walks blocks of
      // 64 chunks from the row's end (the barrier above ordered the stores).
      if (t < 64) {
        double later = 1.0;  // product of the chunks after the current block
        for (int64_t base = ((nch - 1) >> 6) << 6; base >= 0; base -= 64) {
          const int64_t j = base + t;
          const double v = j < nch ? suf[j] : 1.0;
          double below, above, all;
          wave_excl_products(v, &below, &above, &all);
          if (j < nch) suf[j] = above * later;
          later *= all;
        }
      }
      if (t == 0) {
        const int32_t nz = (int32_t)(zeros & 0x7FFFFFFFu);
        const unsigned nf = lds_nf[parity];
        const int32_t nf_col = lds_nf_col[parity];
        lds_nf[parity] = 0u;
        lds_nf_col[parity] = INT32_MAX;
        hdr[r] = ProdHeader{nz, first == INT32_MAX ? -1 : first, (float)pnz,
                            nf == 0u ? -1 : (nf == 1u ? nf_col : -2)};
        // IEEE: the product's sign is the xor of every factor's sign, zeros
        // included; a zero times an infinity or a NaN is NaN.
        const double zero = (zeros >> 31) ? -0.0 : 0.0;
        y[r] = nz > 0 ? (float)(zero * pnz) : (float)pnz;
      }
    }
  }
}

// ------------------------------------------------------------------ backward

// Division of a work-group index by a launch constant d (1 <= d < 2^31),
// exact for every 32-bit dividend, with one multiply-high, a subtraction and
// shifts (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994: the round-down method with an added correction).
// The host computes m, s1 and s2 once per launch.
struct DivMagic {
  uint32_t m, s1, s2;
};
inline DivMagic div_magic(uint32_t d) {
  uint32_t l = 0;  // ceil(log2 d)
  while ((1ull << l) < d) ++l;
  return DivMagic{(uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1), l < 1 ? l : 1u, l > 0 ? l - 1 : 0u};
}
__device__ __forceinline__ uint32_t div_by(uint32_t n, DivMagic q) {
  const uint32_t t = __umulhi(n, q.m);
  return (t + ((n - t) >> q.s1)) >> q.s2;
}


// Product gradient over a flat grid of (row, chunk) tiles, one work-group of
// kProdBlock work-items per tile.  Work-item t holds kProdStripes stripes of
// 4 consecutive columns: stripe s covers columns s * kProdBlock * 4 + 4t ..
// + 3 of the chunk, so every load and store instruction of a wavefront is
// one contiguous kilobyte, and the chunk is the concatenation, in column
// order, of 64 wavefront pieces (stripe-major, then wavefront).
//   Rows with zeros are write-only: row_fill_kernel<Prod> writes them.
//   Zero-free rows: grad[j] = K * P<(j) * P>(j), where K = g * (product of
//   the chunks before) * (product of the chunks after), formed in float64
//   from the forward's saved state, and P<, P> are the exclusive products
//   inside the chunk: inside the work-item (4 columns), over the lanes of the
//   piece (DPP scans), and over the pieces (every wavefront scans the 64
//   piece products from LDS).  No division anywhere.
constexpr int kProdBlock = 1024;
constexpr int kProdWaves = kProdBlock / 64;
constexpr int kProdStripes = (int)(kChunk / (kProdBlock * 4));
static_assert(kProdStripes * kProdWaves == 64, "one wavefront scans the chunk's pieces");

// x of tile (r, k): stripes of 4 consecutive columns, ragged columns as 1.0.
template <bool AL, bool NT>
__device__ __forceinline__ void load_prod_tile(const float* __restrict__ x, int64_t r, int64_t k, int64_t cols,
                                               int t, float (&v)[kProdStripes][4]) {
  const int64_t c0 = k * kChunk;
  const bool full = c0 + kChunk <= cols;
#pragma unroll
  for (int s = 0; s < kProdStripes; ++s)
    load_stripe<AL, NT>(x + r * cols, c0 + ((int64_t)s * kProdBlock + t) * 4, cols, full, 1.0f, v[s]);
}

// Gradient of tile (r, k) of a zero-free row from its x (one barrier:
// every wavefront scans the 64 piece products, which go through `piece`,
// 64 floats of LDS the caller does not reuse before the next barrier).
template <bool AL, bool NT>
__device__ __forceinline__ void prod_tile(const float (&v)[kProdStripes][4], int64_t r, int64_t k, int64_t cols,
                                          int64_t nch, const float* __restrict__ g, const double* __restrict__ pre,
                                          const double* __restrict__ suf, float* __restrict__ grad, float* piece,
                                          int t, int lane, int wave) {
  const int64_t c0 = k * kChunk;
  const bool full = c0 + kChunk <= cols;
  // the rest of the row (chunks before and after), times g, in float64
  const float K = (float)((double)g[r] * pre[r * nch + k] * suf[r * nch + k]);
  float before[kProdStripes], after[kProdStripes];
#pragma unroll
  for (int s = 0; s < kProdStripes; ++s) {
    const float m = (v[s][0] * v[s][1]) * (v[s][2] * v[s][3]);  // this work-item's 4 columns
    float all;
    wave_excl_products(m, &before[s], &after[s], &all);
    if (lane == 0) piece[s * kProdWaves + wave] = all;
  }
  __syncthreads();
  float pb, pa, pall;
  wave_excl_products(piece[lane], &pb, &pa, &pall);
  float* __restrict__ grow = grad + r * cols;
#pragma unroll
  for (int s = 0; s < kProdStripes; ++s) {
    const int pc = s * kProdWaves + wave;  // wavefront-uniform
    const float left = (K * readlane(pb, pc)) * before[s];
    const float right = after[s] * readlane(pa, pc);
    const float p01 = v[s][0] * v[s][1], p23 = v[s][2] * v[s][3];
    float o[4];
    o[0] = left * (v[s][1] * p23) * right;
    o[1] = left * (v[s][0] * p23) * right;
    o[2] = left * (p01 * v[s][3]) * right;
    o[3] = left * (p01 * v[s][2]) * right;
    const int64_t col = c0 + ((int64_t)s * kProdBlock + t) * 4;
    if (col < cols) store_stripe<AL, NT>(grow, col, cols, full, o);
  }
}

// At most 64 VGPRs, so two work-groups fit on a CU (8 wavefronts per SIMD).
// Persistent: work-group w takes the tiles w, w + G, w + 2G, ... (G groups).
// Every wavefront reads the row headers (and g) of 64 of those tiles at once,
// one per lane, so tiles of rows with zeros -- written by
// row_fill_kernel<Prod> -- are skipped at one shared load per 64.  For
// zero-free rows the next tile's x is loaded before the current tile is
// processed (the last tile of a batch of 64 is peeled, so every prefetch is
// unconditional), and a tile needs one barrier: every wavefront scans the 64
// piece products itself.  Used where the tile-counter kernel below does not
// apply.
template <bool AL, bool NT>
__global__ __launch_bounds__(kProdBlock) __attribute__((amdgpu_waves_per_eu(8, 8)))
void row_prod_bwd_kernel(const float* __restrict__ x, const float* __restrict__ g, const void* __restrict__ saved,
                         int64_t rows, int64_t cols, int64_t nch, double inv_nch, float* __restrict__ grad) {
  __shared__ float lds_piece[2][64];  // piece products in column order, one array per tile parity
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const ProdHeader* __restrict__ hdr = (const ProdHeader*)saved;
  const double* __restrict__ pre = prod_prefix((void*)saved, rows);
  const double* __restrict__ suf = prod_suffix((void*)saved, rows, nch);
  const int64_t total = rows * nch, G = gridDim.x;
  const auto row_of = [&](int64_t b) {
    int64_t r = (int64_t)((double)b * inv_nch);  // b / nch, then corrected
    if (r * nch > b) --r;
    if ((r + 1) * nch <= b) ++r;
    return r;
  };
  const auto load_tile = [&](int64_t b, float (&v)[kProdStripes][4]) {
    const int64_t r = row_of(b);
    load_prod_tile<AL, NT>(x, r, b - r * nch, cols, t, v);
  };
  int parity = 0;
  const auto process = [&](int64_t b, const float (&v)[kProdStripes][4]) {
    const int64_t r = row_of(b);
    prod_tile<AL, NT>(v, r, b - r * nch, cols, nch, g, pre, suf, grad, lds_piece[parity], t, lane, wave);
    parity ^= 1;  // the next tile writes the other array: no second barrier
  };
  for (int64_t base = blockIdx.x; base < total; base += 64 * G) {
    // lane j: the zero count of tile base + j * G's row (every wavefront the same)
    const int64_t bj = base + (int64_t)lane * G;
    const bool valid = bj < total;
    int32_t zj = 1;
    if (valid) zj = hdr[row_of(bj)].zeros;
    uint64_t todo = __builtin_amdgcn_ballot_w64(valid && zj == 0);
    if (todo == 0ull) continue;
    // Zero-free rows: the exclusive products, the next tile's x loaded early.
    float cur[kProdStripes][4];
    int64_t b = base + (int64_t)__builtin_ctzll(todo) * G;
    todo &= todo - 1ull;
    load_tile(b, cur);
    while (todo != 0ull) {
      const int64_t bn = base + (int64_t)__builtin_ctzll(todo) * G;
      todo &= todo - 1ull;
      float nxt[kProdStripes][4];
      load_tile(bn, nxt);
      process(b, cur);
#pragma unroll
      for (int s = 0; s < kProdStripes; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) cur[s][e] = nxt[s][e];
      b = bn;
    }
    process(b, cur);
  }
}

// The same gradient with tiles handed out in order by a counter, one per
// grab, to one work-group per CU: the tiles in flight are then neighbours in
// memory, as in a flat launch, while a fixed stride lets work-groups drift
// apart.  Measured on MI355X for 8 GiB of plain read+write (one 1024-wide
// work-group per CU, 4 loads and 4 stores per work-item per tile): strided
// 1.53 ms, counter 1.29 ms, counter in batches of 2 / 4 / 16 tiles per grab
// 1.38 / 1.46 / 1.60 ms, a flat launch 1.31 ms.
//   The zero-free rows come first, as a bitmap in LDS built from the row
// headers (rows <= kDynRows); a launch in which every row holds a zero
// leaves at once, and a tile of a row with zeros costs one grab.  Each
// grab is issued one tile ahead.  ctl[1] is the counter and ctl[2] counts
// the work-groups that finished: the last one re-arms both to zero.
constexpr int64_t kDynRows = 65536;

template <bool AL, bool NT>
__global__ __launch_bounds__(kProdBlock)
void row_prod_bwd_dyn_kernel(const float* __restrict__ x, const float* __restrict__ g,
                             const void* __restrict__ saved, int64_t rows, int64_t cols, int64_t nch, DivMagic dm,
                             float* __restrict__ grad, unsigned* __restrict__ ctl) {
  __shared__ float lds_piece[2][64];
  __shared__ uint32_t lds_zf[kDynRows / 32];  // bit r % 32 of word r / 32: row r has no zero
  __shared__ unsigned lds_tile[2];
  __shared__ int lds_any;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const ProdHeader* __restrict__ hdr = (const ProdHeader*)saved;
  if (t == 0) lds_any = 0;
  __syncthreads();
  bool any = false;
  for (int64_t base = (int64_t)wave * 64; base < rows; base += (int64_t)kProdWaves * 64) {
    const int64_t r = base + lane;
    const uint64_t m = __builtin_amdgcn_ballot_w64(r < rows && hdr[r].zeros == 0);
    if (lane == 0) {  // rows base .. base + 63: words base / 32 and base / 32 + 1
      lds_zf[base >> 5] = (uint32_t)m;
      lds_zf[(base >> 5) + 1] = (uint32_t)(m >> 32);
    }
    any = any || m != 0ull;
  }
  if (any && lane == 0) lds_any = 1;
  __syncthreads();
  if (lds_any != 0) {
    const double* __restrict__ pre = prod_prefix((void*)saved, rows);
    const double* __restrict__ suf = prod_suffix((void*)saved, rows, nch);
    const unsigned total = (unsigned)(rows * nch);  // < 2^31 (the host checks)
    const auto grab = [&]() { return __hip_atomic_fetch_add(ctl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    if (t == 0) lds_tile[0] = grab();
    __syncthreads();
    unsigned b = lds_tile[0];
    int par = 1, parity = 0;
    while (b < total) {
      if (t == 0) lds_tile[par] = grab();  // the next tile, in flight during this one
      const uint32_t r = div_by(b, dm);
      if ((lds_zf[r >> 5] >> (r & 31)) & 1u) {  // the same in every work-item
        const int64_t k = (int64_t)(b - r * (uint32_t)nch);
        float v[kProdStripes][4];
        load_prod_tile<AL, NT>(x, r, k, cols, t, v);
        prod_tile<AL, NT>(v, r, k, cols, nch, g, pre, suf, grad, lds_piece[parity], t, lane, wave);
        parity ^= 1;
      }
      __syncthreads();  // lds_tile[par] written
      b = lds_tile[par];
      par ^= 1;
    }
  }
  if (t == 0) {
    const unsigned prev = __hip_atomic_fetch_add(ctl + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x - 1) {  // every grab of this launch is done
      __hip_atomic_store(ctl + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ctl + 2, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Write-only gradients (sum; min/max; product rows with zeros), one tile of
// kRowBlock x 4 columns per work-group and one 16-byte store per work-item,
// over a flat grid of rows x tiles: for pure writes, many short work-groups
// keep more stores in flight than a persistent loop (measured on MI355X:
// 6.9 TB/s against 6.2 TB/s; product rows with zeros 0.60 ms against 0.96 ms
// for a persistent loop and 0.82 ms inside the exclusive-product kernel).
// The row comes from the work-group index by one multiply-high on the scalar
// unit, so a work-group with nothing to write leaves after a kernel-argument
// load and one header load: with a float64 division and a grid-stride loop
// instead, a zero-free 4096 x 262,144 product matrix took 0.39 ms to
// dispatch and retire its 4 M wavefronts, against 0.22 ms now (a bare
// load-and-leave kernel over the same grid: 0.23 ms).
//   Product rows with zeros: g * (product of the nonzero entries) at the
//   single zero of a row with one; every other column's product of the other
//   entries holds a zero, so it is g * 0 -- or NaN (IEEE 0 * inf) when those
//   other entries hold an infinity or a NaN, which the forward's record of
//   non-finite entries tells.  Work-groups of zero-free rows leave (the
//   exclusive-product kernel writes those rows).
template <Op O, bool AL, bool NT>
__global__ __launch_bounds__(kRowBlock) void row_fill_kernel(const float* __restrict__ g,
                                                             const void* __restrict__ saved, int64_t row0,
                                                             int64_t cols, uint32_t tiles, DivMagic dm,
                                                             float* __restrict__ grad) {
  // The launch covers rows row0 .. row0 + gridDim.x / tiles - 1, tiles work-groups each.
  const uint32_t b = blockIdx.x, rb = div_by(b, dm);
  const int64_t r = row0 + rb;
  const float gr = g[r];
  int64_t hot = -1;
  float hot_val = 0.0f, fill = 0.0f;
  int32_t nonfinite = -1;
  if constexpr (O == Op::Prod) {
    const ProdHeader h = ((const ProdHeader*)saved)[r];
    if (h.zeros == 0) return;  // the same for the whole work-group
    hot = h.zeros == 1 ? h.first_zero : -1;
    hot_val = gr * h.pnz;
    fill = gr * 0.0f;
    nonfinite = h.nonfinite;
  } else if constexpr (O == Op::Sum) {
    fill = gr;
  } else {
    hot = ((const int64_t*)saved)[r];
    hot_val = gr;
  }
  // A writing wavefront waits about 1000-1300 cycles before its store.  The
  // write stream runs faster when each work-group stays resident that much
  // longer (measured on MI355X over a 4096 x 262,144 matrix: sum 636 -> 597,
  // max 638 -> 597, product 625 -> 595 us); past the best length the wait
  // itself limits the rate (product at 22 units: 622 us, at 32: 757 us), and
  // the product's own longer path reaches that point first.
  __builtin_amdgcn_s_sleep(O == Op::Prod ? 16 : 20);
  const int64_t col = (int64_t)(b - rb * tiles) * (kRowBlock * 4) + (int64_t)threadIdx.x * 4;
  if (col >= cols) return;
  float v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool nan_here = nonfinite == -2 || (nonfinite >= 0 && col + e != nonfinite);
    v[e] = (col + e == hot) ? hot_val : (nan_here ? __builtin_nanf("") : fill);
  }
  store_stripe<AL, NT>(grad + r * cols, col, cols, col + 4 <= cols, v);
}

// ------------------------------------------------------------------ host side

size_t rowreduce_saved_bytes(rd_op op, int64_t rows, int64_t cols) {
  switch (op) {
    case RD_SUM: return 0;
    case RD_MAX:
    case RD_MIN: return (size_t)rows * 8;
    case RD_PROD: return (size_t)rows * sizeof(ProdHeader) + (size_t)rows * chunks_of(cols) * 16;
    default: return 0;
  }
}

namespace {
constexpr int64_t kFillBlocks = (int64_t)1 << 22;  // work-groups per fill launch (rows x tiles), at most

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

template <Op O>
hipError_t fwd_op(bool al, int S, const float* x, int64_t rows, int64_t cols, float* y, void* saved, int grid,
                  bool nt, hipStream_t s) {
  return al ? fwd_s<O, true>(S, x, rows, cols, y, saved, grid, nt, s)
            : fwd_s<O, false>(S, x, rows, cols, y, saved, grid, nt, s);
}

template <Op O, bool AL>
hipError_t fill_launch(const float* g, const void* saved, int64_t rows, int64_t cols, float* grad, bool nt,
                       hipStream_t s) {
  const int64_t tiles = (cols + kRowBlock * 4 - 1) / (kRowBlock * 4);  // cols < 2^31: at most 2^21 tiles
  const int64_t per = std::max<int64_t>(1, kFillBlocks / tiles);      // rows per launch
  const DivMagic dm = div_magic((uint32_t)tiles);
  for (int64_t row0 = 0; row0 < rows; row0 += per) {
    const unsigned blocks = (unsigned)(std::min<int64_t>(rows - row0, per) * tiles);
    if (nt) hipLaunchKernelGGL((row_fill_kernel<O, AL, true>), dim3(blocks), dim3(kRowBlock), 0, s, g, saved, row0, cols,
                               (uint32_t)tiles, dm, grad);
    else hipLaunchKernelGGL((row_fill_kernel<O, AL, false>), dim3(blocks), dim3(kRowBlock), 0, s, g, saved, row0, cols,
                            (uint32_t)tiles, dm, grad);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool AL>
hipError_t prod_bwd_launch(const float* x, const float* g, const void* saved, int64_t rows, int64_t cols,
                           float* grad, int groups, bool nt, hipStream_t s) {
  const int64_t nch = chunks_of(cols);
  const int64_t blocks = std::min<int64_t>(rows * nch, (int64_t)groups);  // persistent
  const double inv = 1.0 / (double)nch;
  if (nt) hipLaunchKernelGGL((row_prod_bwd_kernel<AL, true>), dim3((unsigned)blocks), dim3(kProdBlock), 0, s, x, g,
                             saved, rows, cols, nch, inv, grad);
  else hipLaunchKernelGGL((row_prod_bwd_kernel<AL, false>), dim3((unsigned)blocks), dim3(kProdBlock), 0, s, x, g,
                          saved, rows, cols, nch, inv, grad);
  return hipGetLastError();
}

// Product backward: the fill (rows with zeros) and the exclusive products
// (zero-free rows) write disjoint rows, so they may run at once.  With a side
// stream the fill runs there, beside the exclusive-product kernel on the
// caller's stream (one work-group per CU): the fill's work-groups of
// zero-free rows cost their dispatch only (0.22 ms over 4096 x 262,144),
// which then hides behind the exclusive products.  The exclusive-product
// kernel stays on the caller's stream so that it is dispatched first (the
// side stream first waits for the fork): a fill dispatched ahead of it
// crowds the CUs with small work-groups that hold off its 1024-wide ones.
// Measured on MI355X, 4096 x 262,144: every row zero-free 1.84 -> 1.59 ms;
// one zero in every other row 1.19 -> 1.23 ms (1.83 ms with the kernels on
// the other streams); every row with zeros 0.60 -> 0.62 ms (the fork and
// the join).  The caller's stream waits for the side stream before anything
// after the call.
// The exclusive-product kernel on stream s: the tile-counter kernel (one
// work-group per CU) where its counter words are given and its limits hold,
// else the strided one.
template <bool AL>
hipError_t dense_launch(const float* x, const float* g, const void* saved, int64_t rows, int64_t cols,
                        float* grad, int cus, int strided_groups, bool nt, unsigned* dyn_ctl, hipStream_t s) {
  const int64_t nch = chunks_of(cols);
  if (dyn_ctl != nullptr && rows <= kDynRows && rows * nch < ((int64_t)1 << 31)) {
    const DivMagic dm = div_magic((uint32_t)nch);
    if (nt) hipLaunchKernelGGL((row_prod_bwd_dyn_kernel<AL, true>), dim3((unsigned)cus), dim3(kProdBlock), 0, s, x,
                               g, saved, rows, cols, nch, dm, grad, dyn_ctl);
    else hipLaunchKernelGGL((row_prod_bwd_dyn_kernel<AL, false>), dim3((unsigned)cus), dim3(kProdBlock), 0, s, x,
                            g, saved, rows, cols, nch, dm, grad, dyn_ctl);
    return hipGetLastError();
  }
  return prod_bwd_launch<AL>(x, g, saved, rows, cols, grad, strided_groups, nt, s);
}

template <bool AL>
hipError_t prod_bwd(const float* x, const float* g, const void* saved, int64_t rows, int64_t cols, float* grad,
                    int cus, bool nt, hipStream_t s, const SidePath& side, unsigned* dyn_ctl) {
  if (side.stream == nullptr) {
    const hipError_t e = fill_launch<Op::Prod, AL>(g, saved, rows, cols, grad, nt, s);
    if (e != hipSuccess) return e;
    return dense_launch<AL>(x, g, saved, rows, cols, grad, cus, cus * 2, nt, dyn_ctl, s);
  }
  hipError_t e = hipEventRecord(side.fork, s);
  if (e != hipSuccess) return e;
  e = hipStreamWaitEvent(side.stream, side.fork, 0);
  if (e != hipSuccess) return e;
  const hipError_t e_dense = dense_launch<AL>(x, g, saved, rows, cols, grad, cus, cus, nt, dyn_ctl, s);
  const hipError_t e_fill = fill_launch<Op::Prod, AL>(g, saved, rows, cols, grad, nt, side.stream);
  e = hipEventRecord(side.join, side.stream);  // joined whatever the launches returned
  if (e == hipSuccess) e = hipStreamWaitEvent(s, side.join, 0);
  if (e_dense != hipSuccess) return e_dense;
  if (e_fill != hipSuccess) return e_fill;
  return e;
}

template <Op O>
hipError_t bwd_op(bool al, const float* x, const float* g, const void* saved, int64_t rows, int64_t cols,
                  float* grad, int cus, bool nt, hipStream_t s, const SidePath& side, unsigned* dyn_ctl) {
  if constexpr (O == Op::Prod) {
    return al ? prod_bwd<true>(x, g, saved, rows, cols, grad, cus, nt, s, side, dyn_ctl)
              : prod_bwd<false>(x, g, saved, rows, cols, grad, cus, nt, s, side, dyn_ctl);
  } else {
    return al ? fill_launch<O, true>(g, saved, rows, cols, grad, nt, s)
              : fill_launch<O, false>(g, saved, rows, cols, grad, nt, s);
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
                         float* grad, int cus, const Launch& l, hipStream_t s, const SidePath& side,
                         unsigned* dyn_ctl) {
  const bool al = (cols % 4 == 0) && ((uintptr_t)grad % 16 == 0) && (op != RD_PROD || (uintptr_t)x % 16 == 0);
  switch (op) {
    case RD_SUM: return bwd_op<Op::Sum>(al, x, g, saved, rows, cols, grad, cus, l.nontemporal, s, side, dyn_ctl);
    case RD_MAX: return bwd_op<Op::Max>(al, x, g, saved, rows, cols, grad, cus, l.nontemporal, s, side, dyn_ctl);
    case RD_MIN: return bwd_op<Op::Min>(al, x, g, saved, rows, cols, grad, cus, l.nontemporal, s, side, dyn_ctl);
    case RD_PROD: return bwd_op<Op::Prod>(al, x, g, saved, rows, cols, grad, cus, l.nontemporal, s, side, dyn_ctl);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rd
