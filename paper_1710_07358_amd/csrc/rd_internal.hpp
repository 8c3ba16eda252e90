// rd_internal.hpp -- host-side interface between the C ABI (rd_api.cpp) and
// the kernel translation units.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd.h"

namespace rd {

// Launch shape resolved by the host: work-items per group, groups, unroll U
// (16-byte loads in flight per work-item per step), non-temporal loads.
struct Launch {
  int block;
  int grid;
  int unroll;
  bool nontemporal;
  int layout;  // rd_config::layout
  int probe = 0;  // failure-path test: add one bounded wait that runs out (rd_debug_force_wait_timeout)
};

// Device scratch handed to a kernel.  Published values live in tagged
// 64-bit words (one per 32 bits of value); every word is zero between
// launches, and so are the counters.
struct Scratch {
  unsigned* ticket;     // [0]: completion counter; [1]: status (nonzero: a bounded wait ran out, sticky)
  unsigned* counters;   // segmented: one per work-group
  uint64_t* partial;    // kPartialWords words per work-group
  uint64_t* carry;      // segmented: kCarryWords words per slot, 2 slots per work-group
  int64_t partial_cap;  // work-groups
  int64_t carry_cap;    // carry slots
  void* design;         // paper-design baselines: plain partials (kDesignBytes)
  // Scans: control words, per-tile first-head index, published tile and
  // group aggregates (tagged with a launch epoch, so never cleared).
  unsigned* scan_ctl;         // [0] epoch, [1] next tile, [2] arrivals, [3] status (sticky), [4] give-up tag
  uint64_t* scan_tile_first;  // kScanTiles words
  uint64_t* scan_slots;       // kScanSlots x kScanSlotWords words
};

// Scan tiles per call (block x U x V elements each, U = 4 or 8 16-byte
// loads per lane and piece), fan-out and levels of the tree of tile
// aggregates (kScanFan^kScanLevels >= kScanTiles), words per published slot,
// epoch range.
constexpr int64_t kScanTiles = 1 << 19;
constexpr int kScanFanLog = 3;
constexpr int kScanFan = 1 << kScanFanLog;
constexpr int kScanLevels = 7;
constexpr int kScanSlotWords = 2;
constexpr unsigned kScanEpochs = 0x7FFFFFFFu;
// Slots: the group aggregates of every level.
constexpr int64_t scan_slots_total() {
  int64_t total = 0, cap = kScanTiles;
  for (int l = 0; l < kScanLevels; ++l) {
    total += cap;
    cap = (cap + kScanFan - 1) / kScanFan;
  }
  return total;
}
static_assert(kScanLevels * kScanFan <= 64, "one wavefront reads every level at once");
static_assert(((int64_t)1 << (kScanFanLog * kScanLevels)) >= kScanTiles, "tree covers every tile");
constexpr int64_t kScanSlots = scan_slots_total();

constexpr int64_t kDesignBytes = 256 * 1024;

constexpr int kPartialWords = 4;  // up to 16-byte partials (double-double)
constexpr int kCarryWords = 2;    // up to 8-byte accumulators

// Upper bounds the workspace is sized for.
constexpr int kMaxGrid = 8192;
constexpr int kMaxSegWaves = 32768;

using PlainFn = hipError_t (*)(const void* x, int64_t n, void* out, const Scratch& ws,
                               const Launch& l, hipStream_t s);
using SegFn = hipError_t (*)(const void* x, const int64_t* offsets, int64_t nseg, void* out,
                             const Scratch& ws, const Launch& l, hipStream_t s);
using ArgFn = hipError_t (*)(const void* x, int64_t n, void* value_out, int64_t* index_out,
                             const Scratch& ws, const Launch& l, hipStream_t s);

struct ScanCall {
  const void* x;
  int64_t n;
  void* out;
  bool exclusive;
  const int64_t* heads;  // segmented form: run starts, else null
  int64_t nheads;
};
using ScanFn = hipError_t (*)(const ScanCall& c, const Scratch& ws, const Launch& l, hipStream_t s);

// Scan kernels (plain when seg is false), U = 4 or 8.  nullptr when (dt, op)
// is not offered or U has no instantiation.
ScanFn scan_launcher(rd_dtype dt, rd_op op, bool seg, int unroll, bool nontemporal);
ScanFn scan_int(rd_dtype dt, rd_op op, bool seg, int u, bool nt);    // RD_I32 / RD_U32, 32-bit bitwise
ScanFn scan_f32(rd_op op, bool seg, int u, bool nt);
ScanFn scan_f64(rd_op op, bool seg, int u, bool nt);                 // also 64-bit bitwise of float64
ScanFn scan_int64(rd_dtype dt, rd_op op, bool seg, int u, bool nt);  // RD_I64 / RD_U64
ScanFn scan_half(rd_dtype dt, rd_op op, bool seg, int u, bool nt);   // RD_F16 / RD_BF16, 16-bit bitwise

// Arg-reduction (min/max with the lowest index); unroll 2, 4 or 8.
ArgFn arg_launcher(rd_dtype dt, bool is_max, int unroll, bool nontemporal);

// nullptr when (dt, op) is not offered or the unroll has no instantiation
// (plain/compensated: 1, 2, 4, 8, 16; segmented: 2, 4, 8).
PlainFn plain_launcher(rd_dtype dt, rd_op op, int unroll, bool nontemporal);
PlainFn compensated_launcher(rd_dtype dt, int unroll, bool nontemporal);
SegFn segmented_launcher(rd_dtype dt, rd_op op, int unroll, bool nontemporal);

// Per-family instantiations, one translation unit each (parallel builds).
// *_bits32 / *_bits16 / *_bits64: and, or, xor on raw bit patterns.
PlainFn plain_int(rd_dtype dt, rd_op op, int unroll, bool nt);  // RD_I32 / RD_U32
PlainFn plain_bits32(rd_op op, int unroll, bool nt);
PlainFn plain_f32(rd_op op, int unroll, bool nt);
PlainFn plain_f64(rd_op op, int unroll, bool nt);
PlainFn plain_int64(rd_dtype dt, rd_op op, int unroll, bool nt);  // RD_I64 / RD_U64
PlainFn plain_bits64(rd_op op, int unroll, bool nt);
PlainFn plain_half(rd_dtype dt, rd_op op, int unroll, bool nt);  // RD_F16 / RD_BF16, 16-bit bitwise
PlainFn comp_f32(int unroll, bool nt);
PlainFn comp_half(rd_dtype dt, int unroll, bool nt);
SegFn seg_int(rd_dtype dt, rd_op op, int unroll, bool nt);
SegFn seg_bits32(rd_op op, int unroll, bool nt);
SegFn seg_f32(rd_op op, int unroll, bool nt);
SegFn seg_f64(rd_op op, int unroll, bool nt);
SegFn seg_int64(rd_dtype dt, rd_op op, int unroll, bool nt);
SegFn seg_bits64(rd_op op, int unroll, bool nt);
SegFn seg_half(rd_dtype dt, rd_op op, int unroll, bool nt);

// Row-wise forward / backward (float32).  Launch: grid = work-groups per CU
// (capped by rows), unroll = stripes per step (1, 2, 4, 8).
hipError_t rowreduce_fwd(const float* x, int64_t rows, int64_t cols, rd_op op, float* y,
                         void* saved, int cus, const Launch& l, hipStream_t s);
// A second stream of the device and two events: the product backward runs
// its exclusive-product kernel there, beside the fill on the caller's stream
// (fork and join by the events).  Null stream: both run on the caller's.
struct SidePath {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
// dyn_ctl: two words (zero between launches, left zero) for the product's
// tile counter, or null (then the strided kernel runs).
hipError_t rowreduce_bwd(const float* x, const float* g, const void* saved, int64_t rows,
                         int64_t cols, rd_op op, float* grad, int cus, const Launch& l, hipStream_t s,
                         const SidePath& side, unsigned* dyn_ctl);
size_t rowreduce_saved_bytes(rd_op op, int64_t rows, int64_t cols);

// The paper's two designs (sum of int32 / float32), for comparison:
// variant 0 two-stage (Section 2.3), variant 1 unrolled + barrier-free tree
// (Section 3).  partial holds cap elements.
hipError_t paper_design_reduce(const void* x, int64_t n, rd_dtype dt, int variant, int unroll, void* out,
                               void* partial, int cap, int cus, hipStream_t s);

}  // namespace rd
