// rd_api.cpp -- the C ABI declared in include/rd.h: argument validation,
// workspaces, launch-configuration table and dispatch to the kernels.
//
// Launch planning follows Section 2.5 (persistent threads): the grid holds
// only as many work-groups as the device runs at once (blocks_per_cu x CUs),
// capped by the amount of work, and the kernels loop over the data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "rd.h"
#include "rd_internal.hpp"

struct rd_workspace {
  int device;
  void* mem;
  size_t bytes;
  rd::Scratch scratch;
};

namespace {

// A fixed buffer, so that reporting an error never allocates.
thread_local char g_last_error[512];

rd_status fail(rd_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return st;
}

rd_status hip_fail(hipError_t e, const char* what) {
  return fail(RD_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// ---- device properties -----------------------------------------------------

struct DeviceInfo {
  int cus = 0;
  bool ok = false;
};

std::mutex g_mu;
std::map<int, DeviceInfo> g_devices;

rd_status current_device(int* dev, DeviceInfo* info) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceInfo& d = g_devices[*dev];
  if (!d.ok) {
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, *dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    d.cus = cus > 0 ? cus : 1;
    d.ok = true;
  }
  *info = d;
  return RD_OK;
}

// ---- workspaces ------------------------------------------------------------

constexpr size_t kAlign = 256;
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Layout: [ticket, status | per-wavefront counters], partial slots, carry
// slots.  All of it is zero between launches.
size_t counters_bytes() { return round_up(kAlign + (size_t)rd::kMaxSegWaves * 4, kAlign); }
size_t partial_bytes() { return round_up((size_t)rd::kMaxGrid * rd::kPartialWords * 8, kAlign); }
size_t carry_bytes() { return round_up((size_t)rd::kMaxSegWaves * 2 * rd::kCarryWords * 8, kAlign); }
// Scans: control words, per-tile first-head words, tagged slots.
size_t scan_bytes() {
  return kAlign + round_up((size_t)rd::kScanTiles * 8, kAlign) +
         round_up((size_t)rd::kScanSlots * rd::kScanSlotWords * 8, kAlign);
}
size_t workspace_bytes() {
  return counters_bytes() + partial_bytes() + carry_bytes() + (size_t)rd::kDesignBytes + scan_bytes();
}

// Every live workspace (default and explicit), for rd_workspace_status; its
// own lock (workspaces are created while g_mu is held).
std::mutex g_ws_mu;
std::set<rd_workspace*> g_all_ws;

// Set by rd_debug_force_wait_timeout: launches of rd_reduce and rd_scan add
// one bounded wait that runs out.
std::atomic<int> g_probe{0};

rd_status create_workspace(rd_workspace** out, int device) {
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (device != prev && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  rd_workspace* ws = new rd_workspace();
  ws->device = device;
  ws->bytes = workspace_bytes();
  ws->mem = nullptr;
  e = hipMalloc(&ws->mem, ws->bytes);
  if (e == hipSuccess) e = hipMemset(ws->mem, 0, ws->bytes);  // counters and slots start at zero
  if (device != prev) (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    if (ws->mem) (void)hipFree(ws->mem);
    delete ws;
    return e == hipErrorOutOfMemory ? fail(RD_ERR_NOMEM, "workspace: out of device memory")
                                    : hip_fail(e, "workspace allocation");
  }
  char* p = (char*)ws->mem;
  rd::Scratch& s = ws->scratch;
  s.ticket = (unsigned*)p;
  s.counters = (unsigned*)(p + kAlign);
  p += counters_bytes();
  s.partial = (uint64_t*)p;
  s.partial_cap = rd::kMaxGrid;
  p += partial_bytes();
  s.carry = (uint64_t*)p;
  s.carry_cap = (int64_t)rd::kMaxSegWaves * 2;
  p += carry_bytes();
  s.design = p;
  p += rd::kDesignBytes;
  s.scan_ctl = (unsigned*)p;
  p += kAlign;
  s.scan_tile_first = (uint64_t*)p;
  p += round_up((size_t)rd::kScanTiles * 8, kAlign);
  s.scan_slots = (uint64_t*)p;
  {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    g_all_ws.insert(ws);
  }
  *out = ws;
  return RD_OK;
}

std::map<std::pair<int, hipStream_t>, rd_workspace*> g_default_ws;

// create_workspace for callers that go on without one: a failure leaves the
// thread's last-error message as it was.
rd_status create_workspace_quiet(rd_workspace** out, int device) {
  char saved[sizeof(g_last_error)];
  std::memcpy(saved, g_last_error, sizeof(saved));
  const rd_status st = create_workspace(out, device);
  if (st != RD_OK) std::memcpy(g_last_error, saved, sizeof(saved));
  return st;
}

// ---- allocation-free scratch (rd_reduce_noalloc) ---------------------------
//
// One array per GPU, loaded with the library's code object and held until the
// process ends: a 256-byte head (word 0: completion counter, word 1: the
// sticky wait-status word, as in a workspace) followed by the tagged partial
// words of up to kNoAllocGroups work-groups.  The host must never pass the
// array's name to a kernel or a copy (on the host it is only a stand-in): its
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and every use goes through that address.
constexpr int kNoAllocGroups = 4096;
constexpr size_t kNoAllocHeadWords = 32;  // 256 bytes
constexpr size_t kNoAllocWords = kNoAllocHeadWords + (size_t)kNoAllocGroups * rd::kPartialWords;
static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

struct NoAllocDevice {
  bool ready = false;
  int cus = 0;
  uint64_t* ptr = nullptr;  // device address of `scratch` on this device
};
constexpr int kNoAllocMaxDevices = 64;
NoAllocDevice g_noalloc[kNoAllocMaxDevices];  // fixed table: set-up allocates nothing
std::mutex g_noalloc_mu;

// Resolve (once per device) the device address of `scratch` on `dev`, which
// must be the current device.
rd_status noalloc_setup(int dev, NoAllocDevice* out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(RD_ERR_INVALID_ARG, "rd_reduce_noalloc: device %d outside 0..%d", dev, kNoAllocMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocDevice& d = g_noalloc[dev];
  if (!d.ready) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(RD_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    d.cus = cus > 0 ? cus : 1;
    d.ptr = (uint64_t*)p;
    d.ready = true;
  }
  *out = d;
  return RD_OK;
}

// Re-arm the scratch for one launch of `groups` work-groups (plus the probe
// slot): zero the completion counter and the partial slots.  A kernel, not
// hipMemsetAsync, so the call can be captured in a HIP graph; the sticky
// status word is left for rd_workspace_status.
__global__ void noalloc_rearm(uint64_t* words, int64_t partial_words) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ((unsigned*)words)[0] = 0u;
  uint64_t* partial = words + kNoAllocHeadWords;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < partial_words;
       i += (int64_t)gridDim.x * blockDim.x)
    partial[i] = 0ull;
}

// The default workspace of (device, stream) if it exists or can be created
// now (not under graph capture), else null; sets no error.
rd_workspace* default_workspace_quiet(int device, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto key = std::make_pair(device, s);
  auto it = g_default_ws.find(key);
  if (it != g_default_ws.end()) return it->second;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  rd_workspace* w = nullptr;
  if (create_workspace_quiet(&w, device) != RD_OK) return nullptr;
  g_default_ws[key] = w;
  return w;
}

// Resolve the caller's workspace or the default one for (device, stream).
rd_status resolve_workspace(rd_workspace* given, int device, hipStream_t s, rd_workspace** ws) {
  if (given) {
    if (given->device != device)
      return fail(RD_ERR_WORKSPACE, "workspace belongs to device %d, current device is %d",
                  given->device, device);
    *ws = given;
    return RD_OK;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  auto key = std::make_pair(device, s);
  auto it = g_default_ws.find(key);
  if (it != g_default_ws.end()) {
    *ws = it->second;
    return RD_OK;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(RD_ERR_CAPTURE,
                "the default workspace for this stream would be allocated during graph capture; "
                "call once before capturing or pass a workspace");
  rd_workspace* w = nullptr;
  rd_status st = create_workspace(&w, device);
  if (st != RD_OK) return st;
  g_default_ws[key] = w;
  *ws = w;
  return RD_OK;
}

// ---- launch configuration table -------------------------------------------

struct TuneEntry {
  int kind, esize, opclass, lo, hi;  // log2(n) range [lo, hi]
  rd_config cfg;
};

int op_class(rd_op op) {
  if (op == RD_SUM || op == RD_PROD) return 0;
  if (op == RD_MIN || op == RD_MAX) return 1;
  return 2;
}

// Row-wise kinds have no bitwise ops; their class 2 is the product, whose
// forward and backward do different work from the sum's.
int op_class(rd_kind kind, rd_op op) {
  if ((kind == RD_KIND_ROWWISE || kind == RD_KIND_ROWWISE_BWD) && op == RD_PROD) return 2;
  return op_class(op);
}

std::vector<TuneEntry> builtin_table() {
  // Defaults before tuning (measured on MI355X for float32 sums): few
  // resident wavefronts per CU stream best; non-temporal loads and XCD-grouped
  // chunks for inputs far beyond the 256 MB MALL.
  std::vector<TuneEntry> t;
  for (int es : {2, 4, 8})
    for (int oc = 0; oc < 3; ++oc) {
      t.push_back({RD_KIND_PLAIN, es, oc, 0, 17, {256, 2, 4, 0, 0}});
      t.push_back({RD_KIND_PLAIN, es, oc, 18, 23, {256, 4, 2, 0, 1}});
      t.push_back({RD_KIND_PLAIN, es, oc, 24, 62, {512, 2, 2, 1, 1}});
      t.push_back({RD_KIND_COMPENSATED, es, oc, 0, 17, {256, 2, 4, 0, 0}});
      t.push_back({RD_KIND_COMPENSATED, es, oc, 18, 23, {256, 4, 2, 0, 1}});
      t.push_back({RD_KIND_COMPENSATED, es, oc, 24, 62, {256, 8, 1, 1, 1}});
      // segmented: windows of 4 loads per lane (2 for 16-bit data, whose 8 elements per load
      // would otherwise need 32 accumulators), 16 wavefronts per CU
      t.push_back({RD_KIND_SEGMENTED, es, oc, 0, 62, {es == 8 ? 1024 : 512, es == 2 ? 2 : 4, es == 8 ? 1 : 2, 1, 0}});
    }
  // Row-wise (float32), measured at 4096 x 262144: the forward streams best
  // with non-temporal loads, the write-only backward with non-temporal stores.
  t.push_back({RD_KIND_ROWWISE, 4, 0, 0, 62, {256, 2, 4, 1, 0}});
  t.push_back({RD_KIND_ROWWISE, 4, 1, 0, 62, {256, 1, 8, 1, 0}});
  t.push_back({RD_KIND_ROWWISE, 4, 2, 0, 62, {256, 2, 4, 1, 0}});
  t.push_back({RD_KIND_ROWWISE_BWD, 4, 0, 0, 62, {256, 4, 1, 1, 0}});
  t.push_back({RD_KIND_ROWWISE_BWD, 4, 1, 0, 62, {256, 4, 1, 1, 0}});
  t.push_back({RD_KIND_ROWWISE_BWD, 4, 2, 0, 62, {256, 4, 1, 1, 0}});
  // Scans, measured at n = 2^28: large tiles (one 1024-wide work-group per
  // CU, 8 loads per lane and piece) keep the per-tile look-back cost small;
  // segmented scans of 16- and 64-bit data prefer 4 (fewer spilled registers).
  for (int es : {2, 4, 8})
    for (int oc = 0; oc < 3; ++oc) {
      t.push_back({RD_KIND_SCAN, es, oc, 0, 62, {1024, 8, 1, 1, 0}});
      t.push_back({RD_KIND_SEGMENTED_SCAN, es, oc, 0, 62, {1024, es == 4 ? 8 : 4, 1, 1, 0}});
    }
  return t;
}

std::vector<TuneEntry> g_table = builtin_table();
constexpr int kKinds = 7;
bool g_forced[kKinds] = {false, false, false, false, false, false, false};
rd_config g_force_cfg[kKinds];

int log2_ceil(int64_t n) {
  int l = 0;
  while (l < 62 && ((int64_t)1 << l) < n) ++l;
  return l;
}

rd_config choose_config(rd_kind kind, rd_dtype dt, rd_op op, int64_t n) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_forced[kind]) return g_force_cfg[kind];
  const int es = (int)rd_dtype_size(dt), oc = op_class(kind, op), l = log2_ceil(n);
  for (const TuneEntry& e : g_table)
    if (e.kind == (int)kind && e.esize == es && e.opclass == oc && l >= e.lo && l <= e.hi) return e.cfg;
  return rd_config{256, 8, 2, 0, 0};
}

bool valid_config(const rd_config& c) {
  const bool u_ok = c.unroll == 1 || c.unroll == 2 || c.unroll == 4 || c.unroll == 8 || c.unroll == 16;
  return c.block >= 64 && c.block <= 1024 && c.block % 64 == 0 && u_ok && c.blocks_per_cu >= 1 &&
         c.blocks_per_cu <= 64 && (c.nontemporal == 0 || c.nontemporal == 1) && c.layout >= 0 &&
         c.layout <= 2;
}

// Persistent grid: min(work chunks, blocks_per_cu x CUs, workspace capacity).
rd::Launch plan(const rd_config& c, int64_t nvec, int cus, int cap) {
  const int64_t per_chunk = (int64_t)c.block * c.unroll;
  int64_t chunks = (nvec + per_chunk - 1) / per_chunk;
  int64_t g = std::min<int64_t>((int64_t)c.blocks_per_cu * cus, cap);
  g = std::max<int64_t>(1, std::min(g, chunks));
  return rd::Launch{c.block, (int)g, c.unroll, c.nontemporal != 0, c.layout};
}

// Row-wise kernels: 256 work-items; grid carries blocks per CU; unroll is
// the number of stripes per step (1, 2, 4, 8).
rd::Launch row_launch(rd_kind kind, rd_op op, int64_t rows, int64_t cols) {
  const rd_config c = choose_config(kind, RD_F32, op, rows * cols);
  return rd::Launch{256, c.blocks_per_cu, c.unroll > 8 ? 8 : c.unroll, c.nontemporal != 0, c.layout};
}

bool valid_dtype(rd_dtype dt) { return dt >= RD_I32 && dt <= RD_U64; }
bool valid_op(rd_op op) { return op >= RD_SUM && op <= RD_XOR; }

rd_status check_ptr(const void* p, size_t align, const char* name) {
  if (!p) return fail(RD_ERR_INVALID_ARG, "%s is NULL", name);
  if ((uintptr_t)p % align) return fail(RD_ERR_INVALID_ARG, "%s is not aligned to %zu bytes", name, align);
  return RD_OK;
}

}  // namespace

namespace rd {

PlainFn plain_launcher(rd_dtype dt, rd_op op, int unroll, bool nt) {
  switch (dt) {
    case RD_I32:
    case RD_U32: return plain_int(dt, op, unroll, nt);
    case RD_F32: return plain_f32(op, unroll, nt);
    case RD_F64: return plain_f64(op, unroll, nt);
    case RD_F16:
    case RD_BF16: return plain_half(dt, op, unroll, nt);
    case RD_I64:
    case RD_U64: return plain_int64(dt, op, unroll, nt);
  }
  return nullptr;
}

PlainFn compensated_launcher(rd_dtype dt, int unroll, bool nt) {
  switch (dt) {
    case RD_F32: return comp_f32(unroll, nt);
    case RD_F16:
    case RD_BF16: return comp_half(dt, unroll, nt);
    default: return nullptr;
  }
}

SegFn segmented_launcher(rd_dtype dt, rd_op op, int unroll, bool nt) {
  switch (dt) {
    case RD_I32:
    case RD_U32: return seg_int(dt, op, unroll, nt);
    case RD_F32: return seg_f32(op, unroll, nt);
    case RD_F64: return seg_f64(op, unroll, nt);
    case RD_F16:
    case RD_BF16: return seg_half(dt, op, unroll, nt);
    case RD_I64:
    case RD_U64: return seg_int64(dt, op, unroll, nt);
  }
  return nullptr;
}

ScanFn scan_launcher(rd_dtype dt, rd_op op, bool seg, int u, bool nt) {
  const bool bitwise = (op == RD_AND || op == RD_OR || op == RD_XOR);
  switch (dt) {
    case RD_I32:
    case RD_U32: return scan_int(dt, op, seg, u, nt);
    case RD_F32: return bitwise ? scan_int(RD_U32, op, seg, u, nt) : scan_f32(op, seg, u, nt);
    case RD_F64: return bitwise ? scan_int64(RD_U64, op, seg, u, nt) : scan_f64(op, seg, u, nt);
    case RD_F16:
    case RD_BF16: return scan_half(dt, op, seg, u, nt);
    case RD_I64:
    case RD_U64: return scan_int64(dt, op, seg, u, nt);
  }
  return nullptr;
}

}  // namespace rd

namespace {

// Shared body of rd_scan and rd_segmented_scan.
rd_status scan_call(const char* name, const void* x, int64_t n, const int64_t* heads, int64_t nheads, bool seg,
                    rd_dtype dt, rd_op op, int exclusive, void* out, rd_workspace* ws, void* stream) {
  if (!valid_dtype(dt)) return fail(RD_ERR_INVALID_ARG, "%s: invalid dtype %d", name, (int)dt);
  if (!valid_op(op)) return fail(RD_ERR_INVALID_ARG, "%s: invalid op %d", name, (int)op);
  if (n < 0) return fail(RD_ERR_INVALID_ARG, "%s: n = %lld < 0", name, (long long)n);
  if (nheads < 0 || nheads >= ((int64_t)1 << 31))
    return fail(RD_ERR_INVALID_ARG, "%s: noffsets = %lld outside [0, 2^31)", name, (long long)nheads);
  if (n == 0) return RD_OK;
  const size_t es = rd_dtype_size(dt);
  rd_dtype odt;
  rd_out_dtype(dt, op, &odt);
  rd_status st;
  if ((st = check_ptr(x, es, "x")) != RD_OK) return st;
  if ((st = check_ptr(out, rd_dtype_size(odt), "out")) != RD_OK) return st;
  if (seg && nheads > 0 && (st = check_ptr(heads, 8, "offsets")) != RD_OK) return st;
  int dev;
  DeviceInfo info;
  if ((st = current_device(&dev, &info)) != RD_OK) return st;
  rd_workspace* w;
  if ((st = resolve_workspace(ws, dev, (hipStream_t)stream, &w)) != RD_OK) return st;
  const rd_config cfg = choose_config(seg ? RD_KIND_SEGMENTED_SCAN : RD_KIND_SCAN, dt, op, n);
  const int unroll = cfg.unroll >= 8 ? 8 : 4;  // the instantiated tile depths
  const int64_t tile = (int64_t)cfg.block * unroll * (int64_t)(16 / es);
  const int64_t ntiles = (n + tile - 1) / tile;
  if (ntiles > rd::kScanTiles)
    return fail(RD_ERR_INVALID_ARG, "%s: n = %lld needs %lld tiles of %lld elements; at most %lld per call", name,
                (long long)n, (long long)ntiles, (long long)tile, (long long)rd::kScanTiles);
  rd::ScanFn fn = rd::scan_launcher(dt, op, seg, unroll, cfg.nontemporal != 0);
  if (!fn) return fail(RD_ERR_UNSUPPORTED, "%s: no kernel for dtype %d op %d", name, (int)dt, (int)op);
  rd::Launch l{cfg.block, std::max(1, cfg.blocks_per_cu * info.cus), unroll, cfg.nontemporal != 0, 0};
  l.probe = g_probe.load();
  const rd::ScanCall c{x, n, out, exclusive != 0, seg ? heads : nullptr, seg ? nheads : 0};
  hipError_t e = fn(c, w->scratch, l, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, name);
}

}  // namespace

extern "C" {

// ---- side stream of the product backward ----------------------------------

// Per device: a second stream (default priority, non-blocking) and two events
// for the product backward's fork and join, created once and kept until the
// process ends.  The mutex keeps one caller's record / wait / launch / record
// / wait sequence whole, so concurrent callers never wait on each other's
// event records.  If creation fails the backward runs both kernels on the
// caller's stream.
constexpr int kSideMaxDevices = 64;
struct SideDevice {
  std::mutex mu;
  bool tried = false;
  rd::SidePath path;
};
SideDevice g_side[kSideMaxDevices];

// With ss.mu held.
void side_setup(SideDevice& ss) {
  if (ss.tried) return;
  ss.tried = true;
  rd::SidePath p;
  if (hipStreamCreateWithFlags(&p.stream, hipStreamNonBlocking) != hipSuccess) p.stream = nullptr;
  if (p.stream && (hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) != hipSuccess ||
                   hipEventCreateWithFlags(&p.join, hipEventDisableTiming) != hipSuccess)) {
    if (p.fork) (void)hipEventDestroy(p.fork);
    if (p.join) (void)hipEventDestroy(p.join);
    (void)hipStreamDestroy(p.stream);
    p = rd::SidePath{};
  }
  ss.path = p;
}

rd_status rd_init(void) {
  int dev;
  DeviceInfo info;
  rd_status st = current_device(&dev, &info);
  if (st != RD_OK) return st;
  NoAllocDevice d;
  if ((st = noalloc_setup(dev, &d)) != RD_OK) return st;
  if (dev >= 0 && dev < kSideMaxDevices) {
    std::lock_guard<std::mutex> lock(g_side[dev].mu);
    side_setup(g_side[dev]);
  }
  return RD_OK;
}

size_t rd_dtype_size(rd_dtype dt) {
  switch (dt) {
    case RD_I32: case RD_U32: case RD_F32: return 4;
    case RD_F64: case RD_I64: case RD_U64: return 8;
    case RD_F16: case RD_BF16: return 2;
  }
  return 0;
}

rd_status rd_out_dtype(rd_dtype dt, rd_op op, rd_dtype* out) {
  if (!valid_dtype(dt) || !valid_op(op) || !out) return fail(RD_ERR_INVALID_ARG, "rd_out_dtype: bad argument");
  *out = ((dt == RD_F16 || dt == RD_BF16) && (op == RD_SUM || op == RD_PROD)) ? RD_F32 : dt;
  return RD_OK;
}

rd_status rd_workspace_create(rd_workspace** ws, int device) {
  if (!ws) return fail(RD_ERR_INVALID_ARG, "rd_workspace_create: ws is NULL");
  return create_workspace(ws, device);
}

rd_status rd_workspace_destroy(rd_workspace* ws) {
  if (!ws) return RD_OK;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto it = g_default_ws.begin(); it != g_default_ws.end(); ++it)
      if (it->second == ws) return fail(RD_ERR_INVALID_ARG, "cannot destroy a default workspace");
  }
  {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    g_all_ws.erase(ws);
  }
  hipError_t e = hipFree(ws->mem);
  delete ws;
  return e == hipSuccess ? RD_OK : hip_fail(e, "hipFree");
}

rd_status rd_workspace_status(rd_workspace* ws, unsigned* flags) {
  if (!flags) return fail(RD_ERR_INVALID_ARG, "rd_workspace_status: flags is NULL");
  int dev;
  DeviceInfo info;
  rd_status st = current_device(&dev, &info);
  if (st != RD_OK) return st;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "rd_workspace_status: hipDeviceSynchronize");
  std::vector<rd_workspace*> targets;
  if (ws) {
    if (ws->device != dev)
      return fail(RD_ERR_WORKSPACE, "workspace belongs to device %d, current device is %d", ws->device, dev);
    targets.push_back(ws);
  } else {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    for (rd_workspace* w : g_all_ws)
      if (w->device == dev) targets.push_back(w);
  }
  unsigned f = 0;
  const unsigned zero = 0;
  for (rd_workspace* w : targets) {
    unsigned grid_word = 0, scan_word = 0;
    if ((e = hipMemcpy(&grid_word, w->scratch.ticket + 1, 4, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(&scan_word, w->scratch.scan_ctl + 3, 4, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "rd_workspace_status: read");
    if (grid_word) f |= RD_WAIT_GRID;
    if (scan_word) f |= RD_WAIT_SCAN;
    if ((grid_word && (e = hipMemcpy(w->scratch.ticket + 1, &zero, 4, hipMemcpyHostToDevice)) != hipSuccess) ||
        (scan_word && (e = hipMemcpy(w->scratch.scan_ctl + 3, &zero, 4, hipMemcpyHostToDevice)) != hipSuccess))
      return hip_fail(e, "rd_workspace_status: clear");
  }
  if (!ws && dev >= 0 && dev < kNoAllocMaxDevices) {  // the allocation-free scratch of this device
    NoAllocDevice d;
    {
      std::lock_guard<std::mutex> lock(g_noalloc_mu);
      d = g_noalloc[dev];
    }
    if (d.ready) {
      unsigned* status = (unsigned*)d.ptr + 1;
      unsigned word = 0;
      if ((e = hipMemcpy(&word, status, 4, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "rd_workspace_status: read");
      if (word) {
        f |= RD_WAIT_GRID;
        if ((e = hipMemcpy(status, &zero, 4, hipMemcpyHostToDevice)) != hipSuccess)
          return hip_fail(e, "rd_workspace_status: clear");
      }
    }
  }
  *flags = f;
  return RD_OK;
}

rd_status rd_debug_force_wait_timeout(int on) {
  g_probe.store(on ? 1 : 0);
  return RD_OK;
}

rd_status rd_workspace_reset(rd_workspace* ws, void* stream) {
  if (!ws) return fail(RD_ERR_INVALID_ARG, "rd_workspace_reset: ws is NULL");
  hipError_t e = hipMemsetAsync(ws->mem, 0, ws->bytes, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, "hipMemsetAsync");
}

rd_status rd_reduce(const void* x, int64_t n, rd_dtype dt, rd_op op, void* out, rd_workspace* ws,
                    void* stream) {
  if (!valid_dtype(dt)) return fail(RD_ERR_INVALID_ARG, "rd_reduce: invalid dtype %d", (int)dt);
  if (!valid_op(op)) return fail(RD_ERR_INVALID_ARG, "rd_reduce: invalid op %d", (int)op);
  if (n < 0) return fail(RD_ERR_INVALID_ARG, "rd_reduce: n = %lld < 0", (long long)n);
  const size_t es = rd_dtype_size(dt);
  rd_dtype odt;
  rd_out_dtype(dt, op, &odt);
  rd_status st;
  if (n > 0 && (st = check_ptr(x, es, "x")) != RD_OK) return st;
  if ((st = check_ptr(out, rd_dtype_size(odt), "out")) != RD_OK) return st;
  int dev;
  DeviceInfo info;
  if ((st = current_device(&dev, &info)) != RD_OK) return st;
  rd_workspace* w;
  if ((st = resolve_workspace(ws, dev, (hipStream_t)stream, &w)) != RD_OK) return st;
  const rd_config cfg = choose_config(RD_KIND_PLAIN, dt, op, n);
  rd::PlainFn fn = rd::plain_launcher(dt, op, cfg.unroll, cfg.nontemporal != 0);
  if (!fn) return fail(RD_ERR_UNSUPPORTED, "rd_reduce: no kernel for dtype %d op %d unroll %d", (int)dt, (int)op, cfg.unroll);
  const int probe = g_probe.load();
  // With the probe on, slot G (one past the grid) must exist: cap the grid one lower.
  rd::Launch l = plan(cfg, (n * (int64_t)es) / 16, info.cus, (int)w->scratch.partial_cap - probe);
  l.probe = probe;
  hipError_t e = fn(n > 0 ? x : out, n, out, w->scratch, l, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, "rd_reduce launch");
}

rd_status rd_reduce_noalloc(const void* x, int64_t n, rd_dtype dt, rd_op op, void* out, void* stream) {
  if (!valid_dtype(dt)) return fail(RD_ERR_INVALID_ARG, "rd_reduce_noalloc: invalid dtype %d", (int)dt);
  if (!valid_op(op)) return fail(RD_ERR_INVALID_ARG, "rd_reduce_noalloc: invalid op %d", (int)op);
  if (n < 0) return fail(RD_ERR_INVALID_ARG, "rd_reduce_noalloc: n = %lld < 0", (long long)n);
  const size_t es = rd_dtype_size(dt);
  rd_dtype odt;
  rd_out_dtype(dt, op, &odt);
  rd_status st;
  if (n > 0 && (st = check_ptr(x, es, "x")) != RD_OK) return st;
  if ((st = check_ptr(out, rd_dtype_size(odt), "out")) != RD_OK) return st;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  NoAllocDevice d;
  if ((st = noalloc_setup(dev, &d)) != RD_OK) return st;
  const rd_config cfg = choose_config(RD_KIND_PLAIN, dt, op, n);
  rd::PlainFn fn = rd::plain_launcher(dt, op, cfg.unroll, cfg.nontemporal != 0);
  if (!fn)
    return fail(RD_ERR_UNSUPPORTED, "rd_reduce_noalloc: no kernel for dtype %d op %d unroll %d", (int)dt, (int)op,
                cfg.unroll);
  const int probe = g_probe.load();
  rd::Launch l = plan(cfg, (n * (int64_t)es) / 16, d.cus, kNoAllocGroups - probe);
  l.probe = probe;
  // The grid is capped at the scratch's capacity above (the kernel loops over
  // any n), so this cannot trigger; it guards the scratch bound itself.
  if (l.grid < 1 || l.grid + probe > kNoAllocGroups)
    return fail(RD_ERR_INVALID_ARG, "rd_reduce_noalloc: %d work-groups exceed the scratch's %d", l.grid,
                kNoAllocGroups);
  rd::Scratch sc{};
  sc.ticket = (unsigned*)d.ptr;
  sc.partial = d.ptr + kNoAllocHeadWords;
  sc.partial_cap = kNoAllocGroups;
  const int64_t words = (int64_t)(l.grid + probe) * rd::kPartialWords;
  hipLaunchKernelGGL(noalloc_rearm, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d.ptr,
                     words);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "rd_reduce_noalloc: re-arm launch");
  e = fn(n > 0 ? x : out, n, out, sc, l, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, "rd_reduce_noalloc launch");
}

rd_status rd_reduce_compensated(const void* x, int64_t n, rd_dtype dt, double* out, rd_workspace* ws,
                                void* stream) {
  if (!valid_dtype(dt)) return fail(RD_ERR_INVALID_ARG, "rd_reduce_compensated: invalid dtype %d", (int)dt);
  if (dt != RD_F32 && dt != RD_F16 && dt != RD_BF16)
    return fail(RD_ERR_UNSUPPORTED, "rd_reduce_compensated: dtype %d (float32, float16, bfloat16 only)", (int)dt);
  if (n < 0) return fail(RD_ERR_INVALID_ARG, "rd_reduce_compensated: n < 0");
  const size_t es = rd_dtype_size(dt);
  rd_status st;
  if (n > 0 && (st = check_ptr(x, es, "x")) != RD_OK) return st;
  if ((st = check_ptr(out, 8, "out")) != RD_OK) return st;
  int dev;
  DeviceInfo info;
  if ((st = current_device(&dev, &info)) != RD_OK) return st;
  rd_workspace* w;
  if ((st = resolve_workspace(ws, dev, (hipStream_t)stream, &w)) != RD_OK) return st;
  const rd_config cfg = choose_config(RD_KIND_COMPENSATED, dt, RD_SUM, n);
  rd::PlainFn fn = rd::compensated_launcher(dt, cfg.unroll, cfg.nontemporal != 0);
  if (!fn) return fail(RD_ERR_UNSUPPORTED, "rd_reduce_compensated: no kernel for unroll %d", cfg.unroll);
  const rd::Launch l = plan(cfg, (n * (int64_t)es) / 16, info.cus, (int)w->scratch.partial_cap);
  hipError_t e = fn(n > 0 ? x : (const void*)out, n, out, w->scratch, l, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, "rd_reduce_compensated launch");
}

rd_status rd_segmented_reduce(const void* x, const int64_t* offsets, int64_t nseg, rd_dtype dt, rd_op op,
                              void* out, rd_workspace* ws, void* stream) {
  if (!valid_dtype(dt)) return fail(RD_ERR_INVALID_ARG, "rd_segmented_reduce: invalid dtype %d", (int)dt);
  if (!valid_op(op)) return fail(RD_ERR_INVALID_ARG, "rd_segmented_reduce: invalid op %d", (int)op);
  if (nseg < 0) return fail(RD_ERR_INVALID_ARG, "rd_segmented_reduce: nseg < 0");
  if (nseg == 0) return RD_OK;
  const size_t es = rd_dtype_size(dt);
  rd_dtype odt;
  rd_out_dtype(dt, op, &odt);
  rd_status st;
  if ((st = check_ptr(x, es, "x")) != RD_OK) return st;
  if ((st = check_ptr(offsets, 8, "offsets")) != RD_OK) return st;
  if ((st = check_ptr(out, rd_dtype_size(odt), "out")) != RD_OK) return st;
  int dev;
  DeviceInfo info;
  if ((st = current_device(&dev, &info)) != RD_OK) return st;
  rd_workspace* w;
  if ((st = resolve_workspace(ws, dev, (hipStream_t)stream, &w)) != RD_OK) return st;
  const rd_config cfg = choose_config(RD_KIND_SEGMENTED, dt, op, (int64_t)1 << 28);
  rd::SegFn fn = rd::segmented_launcher(dt, op, cfg.unroll, cfg.nontemporal != 0);
  if (!fn) return fail(RD_ERR_UNSUPPORTED, "rd_segmented_reduce: no kernel for dtype %d op %d", (int)dt, (int)op);
  // The element count lives on the device (offsets[nseg]); the grid is the
  // persistent maximum and the kernel divides the range it reads.
  const int waves_per_block = cfg.block / 64;
  int grid = std::min(cfg.blocks_per_cu * info.cus, rd::kMaxSegWaves / waves_per_block);
  grid = std::max(grid, 1);
  const rd::Launch l{cfg.block, grid, cfg.unroll, cfg.nontemporal != 0, cfg.layout};
  hipError_t e = fn(x, offsets, nseg, out, w->scratch, l, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, "rd_segmented_reduce launch");
}

rd_status rd_argreduce(const void* x, int64_t n, rd_dtype dt, rd_op op, void* value_out, int64_t* index_out,
                       rd_workspace* ws, void* stream) {
  if (!valid_dtype(dt)) return fail(RD_ERR_INVALID_ARG, "rd_argreduce: invalid dtype %d", (int)dt);
  if (op != RD_MIN && op != RD_MAX) return fail(RD_ERR_UNSUPPORTED, "rd_argreduce: op must be RD_MIN or RD_MAX");
  if (n < 0) return fail(RD_ERR_INVALID_ARG, "rd_argreduce: n < 0");
  const size_t es = rd_dtype_size(dt);
  rd_status st;
  if (n > 0 && (st = check_ptr(x, es, "x")) != RD_OK) return st;
  if ((st = check_ptr(value_out, es, "value_out")) != RD_OK) return st;
  if ((st = check_ptr(index_out, 8, "index_out")) != RD_OK) return st;
  int dev;
  DeviceInfo info;
  if ((st = current_device(&dev, &info)) != RD_OK) return st;
  rd_workspace* w;
  if ((st = resolve_workspace(ws, dev, (hipStream_t)stream, &w)) != RD_OK) return st;
  rd_config cfg = choose_config(RD_KIND_PLAIN, dt, op, n);
  cfg.unroll = cfg.unroll < 2 ? 2 : (cfg.unroll > 8 ? 8 : cfg.unroll);
  rd::ArgFn fn = rd::arg_launcher(dt, op == RD_MAX, cfg.unroll, cfg.nontemporal != 0);
  if (!fn) return fail(RD_ERR_UNSUPPORTED, "rd_argreduce: no kernel for dtype %d", (int)dt);
  const rd::Launch l = plan(cfg, (n * (int64_t)es) / 16, info.cus, (int)w->scratch.partial_cap);
  hipError_t e = fn(n > 0 ? x : value_out, n, value_out, index_out, w->scratch, l, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, "rd_argreduce launch");
}

rd_status rd_reduce_paper_design(const void* x, int64_t n, rd_dtype dt, int variant, int unroll, void* out,
                                 rd_workspace* ws, void* stream) {
  if (dt != RD_F32 && dt != RD_I32)
    return fail(RD_ERR_UNSUPPORTED, "rd_reduce_paper_design: int32 or float32 only");
  if (variant != 0 && variant != 1) return fail(RD_ERR_INVALID_ARG, "rd_reduce_paper_design: variant 0 or 1");
  const bool f_ok = unroll >= 1 && (unroll <= 8 || unroll == 16);
  if ((variant == 0 && unroll != 1) || !f_ok)
    return fail(RD_ERR_INVALID_ARG, "rd_reduce_paper_design: unroll %d (variant 0: 1; variant 1: 1..8 or 16)", unroll);
  if (n < 0) return fail(RD_ERR_INVALID_ARG, "rd_reduce_paper_design: n < 0");
  rd_status st;
  if (n > 0 && (st = check_ptr(x, 4, "x")) != RD_OK) return st;
  if ((st = check_ptr(out, 4, "out")) != RD_OK) return st;
  int dev;
  DeviceInfo info;
  if ((st = current_device(&dev, &info)) != RD_OK) return st;
  rd_workspace* w;
  if ((st = resolve_workspace(ws, dev, (hipStream_t)stream, &w)) != RD_OK) return st;
  hipError_t e = rd::paper_design_reduce(n > 0 ? x : out, n, dt, variant, unroll, out, w->scratch.design,
                                         (int)(rd::kDesignBytes / 4), info.cus, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, "rd_reduce_paper_design launch");
}

rd_status rd_scan(const void* x, int64_t n, rd_dtype dt, rd_op op, int exclusive, void* out, rd_workspace* ws,
                  void* stream) {
  return scan_call("rd_scan", x, n, nullptr, 0, false, dt, op, exclusive, out, ws, stream);
}

rd_status rd_segmented_scan(const void* x, int64_t n, const int64_t* offsets, int64_t noffsets, rd_dtype dt,
                            rd_op op, int exclusive, void* out, rd_workspace* ws, void* stream) {
  return scan_call("rd_segmented_scan", x, n, offsets, noffsets, true, dt, op, exclusive, out, ws, stream);
}

size_t rd_saved_bytes(rd_op op, int64_t rows, int64_t cols) {
  if (rows < 0 || cols < 0) return 0;
  return rd::rowreduce_saved_bytes(op, rows, cols);
}

rd_status rd_rowreduce_fwd(const void* x, int64_t rows, int64_t cols, rd_dtype dt, rd_op op, void* y,
                           void* saved, void* stream) {
  if (dt != RD_F32) return fail(RD_ERR_UNSUPPORTED, "rd_rowreduce_fwd: float32 only");
  if (op != RD_SUM && op != RD_MAX && op != RD_MIN && op != RD_PROD)
    return fail(RD_ERR_UNSUPPORTED, "rd_rowreduce_fwd: op %d (sum, max, min, prod only)", (int)op);
  if (rows < 0 || cols < 0) return fail(RD_ERR_INVALID_ARG, "rd_rowreduce_fwd: negative shape");
  if (cols > INT32_MAX) return fail(RD_ERR_INVALID_ARG, "rd_rowreduce_fwd: cols > 2^31 - 1");
  if (rows == 0) return RD_OK;
  rd_status st;
  if (cols > 0 && (st = check_ptr(x, 4, "x")) != RD_OK) return st;
  if ((st = check_ptr(y, 4, "y")) != RD_OK) return st;
  if (op != RD_SUM && (st = check_ptr(saved, 8, "saved")) != RD_OK) return st;
  int dev;
  DeviceInfo info;
  if ((st = current_device(&dev, &info)) != RD_OK) return st;
  const rd::Launch l = row_launch(RD_KIND_ROWWISE, op, rows, cols);
  hipError_t e = rd::rowreduce_fwd((const float*)x, rows, cols, op, (float*)y, saved, info.cus, l, (hipStream_t)stream);
  return e == hipSuccess ? RD_OK : hip_fail(e, "rd_rowreduce_fwd launch");
}

rd_status rd_rowreduce_bwd(const void* x, const void* g, const void* saved, int64_t rows, int64_t cols,
                           rd_dtype dt, rd_op op, void* grad_in, void* stream) {
  if (dt != RD_F32) return fail(RD_ERR_UNSUPPORTED, "rd_rowreduce_bwd: float32 only");
  if (op != RD_SUM && op != RD_MAX && op != RD_MIN && op != RD_PROD)
    return fail(RD_ERR_UNSUPPORTED, "rd_rowreduce_bwd: op %d (sum, max, min, prod only)", (int)op);
  if (rows < 0 || cols < 0) return fail(RD_ERR_INVALID_ARG, "rd_rowreduce_bwd: negative shape");
  if (cols > INT32_MAX) return fail(RD_ERR_INVALID_ARG, "rd_rowreduce_bwd: cols > 2^31 - 1");
  if (rows == 0 || cols == 0) return RD_OK;
  rd_status st;
  if ((st = check_ptr(g, 4, "g")) != RD_OK) return st;
  if ((st = check_ptr(grad_in, 4, "grad_in")) != RD_OK) return st;
  if (op != RD_SUM && (st = check_ptr(saved, 8, "saved")) != RD_OK) return st;
  if (op == RD_PROD && (st = check_ptr(x, 4, "x")) != RD_OK) return st;
  int dev;
  DeviceInfo info;
  if ((st = current_device(&dev, &info)) != RD_OK) return st;
  const rd::Launch l = row_launch(RD_KIND_ROWWISE_BWD, op, rows, cols);
  hipError_t e;
  if (op == RD_PROD && dev >= 0 && dev < kSideMaxDevices) {
    // The exclusive-product kernel's tile counter: the scan's counter words of
    // the stream's default workspace (zero between launches; the same stream
    // orders every user of them).
    rd_workspace* w = default_workspace_quiet(dev, (hipStream_t)stream);
    unsigned* dyn_ctl = w ? w->scratch.scan_ctl : nullptr;
    SideDevice& ss = g_side[dev];
    std::lock_guard<std::mutex> lock(ss.mu);
    side_setup(ss);
    e = rd::rowreduce_bwd((const float*)x, (const float*)g, saved, rows, cols, op, (float*)grad_in, info.cus, l,
                          (hipStream_t)stream, ss.path, dyn_ctl);
  } else {
    e = rd::rowreduce_bwd((const float*)x, (const float*)g, saved, rows, cols, op, (float*)grad_in, info.cus, l,
                          (hipStream_t)stream, rd::SidePath{}, nullptr);
  }
  return e == hipSuccess ? RD_OK : hip_fail(e, "rd_rowreduce_bwd launch");
}

rd_status rd_config_get(rd_kind kind, rd_dtype dt, rd_op op, int64_t n, rd_config* cfg) {
  if (!cfg || kind < RD_KIND_PLAIN || kind > RD_KIND_SEGMENTED_SCAN || !valid_dtype(dt) || !valid_op(op))
    return fail(RD_ERR_INVALID_ARG, "rd_config_get: bad argument");
  *cfg = choose_config(kind, dt, op, n);
  return RD_OK;
}

rd_status rd_config_force(rd_kind kind, const rd_config* cfg) {
  if (kind < RD_KIND_PLAIN || kind > RD_KIND_SEGMENTED_SCAN) return fail(RD_ERR_INVALID_ARG, "rd_config_force: bad kind");
  if (cfg && !valid_config(*cfg))
    return fail(RD_ERR_INVALID_ARG, "rd_config_force: block %d unroll %d blocks_per_cu %d nontemporal %d layout %d",
                cfg->block, cfg->unroll, cfg->blocks_per_cu, cfg->nontemporal, cfg->layout);
  std::lock_guard<std::mutex> lock(g_mu);
  g_forced[kind] = cfg != nullptr;
  if (cfg) g_force_cfg[kind] = *cfg;
  return RD_OK;
}

rd_status rd_tune_load(const char* path) {
  if (!path) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_table = builtin_table();
    return RD_OK;
  }
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(RD_ERR_INVALID_ARG, "rd_tune_load: cannot open %s", path);
  std::vector<TuneEntry> t;
  char line[512];
  int lineno = 0;
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    char* hash = std::strchr(line, '#');
    if (hash) *hash = 0;
    TuneEntry e;
    int k = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d", &e.kind, &e.esize, &e.opclass, &e.lo, &e.hi,
                        &e.cfg.block, &e.cfg.unroll, &e.cfg.blocks_per_cu, &e.cfg.nontemporal, &e.cfg.layout);
    if (k <= 0) continue;
    if (k != 10 || e.kind < 0 || e.kind >= kKinds || !valid_config(e.cfg)) {
      std::fclose(f);
      return fail(RD_ERR_INVALID_ARG, "rd_tune_load: %s:%d: malformed entry", path, lineno);
    }
    t.push_back(e);
  }
  std::fclose(f);
  // Entries not covered by the file keep the built-in defaults (appended last,
  // so file entries take precedence).
  std::vector<TuneEntry> d = builtin_table();
  t.insert(t.end(), d.begin(), d.end());
  std::lock_guard<std::mutex> lock(g_mu);
  g_table = t;
  return RD_OK;
}

const char* rd_last_error(void) { return g_last_error; }

}  // extern "C"
