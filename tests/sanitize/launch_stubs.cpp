// Stand-ins for the kernel translation units, so the C ABI's host code can be
// built and run under a host sanitizer without a GPU: every launcher lookup
// finds no kernel and every launch reports an error.
#include "rd_internal.hpp"

namespace rd {
ScanFn scan_int(rd_dtype, rd_op, bool, int, bool) { return nullptr; }
ScanFn scan_f32(rd_op, bool, int, bool) { return nullptr; }
ScanFn scan_f64(rd_op, bool, int, bool) { return nullptr; }
ScanFn scan_int64(rd_dtype, rd_op, bool, int, bool) { return nullptr; }
ScanFn scan_half(rd_dtype, rd_op, bool, int, bool) { return nullptr; }
ArgFn arg_launcher(rd_dtype, bool, int, bool) { return nullptr; }
PlainFn plain_int(rd_dtype, rd_op, int, bool) { return nullptr; }
PlainFn plain_bits32(rd_op, int, bool) { return nullptr; }
PlainFn plain_f32(rd_op, int, bool) { return nullptr; }
PlainFn plain_f64(rd_op, int, bool) { return nullptr; }
PlainFn plain_int64(rd_dtype, rd_op, int, bool) { return nullptr; }
PlainFn plain_bits64(rd_op, int, bool) { return nullptr; }
PlainFn plain_half(rd_dtype, rd_op, int, bool) { return nullptr; }
PlainFn comp_f32(int, bool) { return nullptr; }
PlainFn comp_half(rd_dtype, int, bool) { return nullptr; }
SegFn seg_int(rd_dtype, rd_op, int, bool) { return nullptr; }
SegFn seg_bits32(rd_op, int, bool) { return nullptr; }
SegFn seg_f32(rd_op, int, bool) { return nullptr; }
SegFn seg_f64(rd_op, int, bool) { return nullptr; }
SegFn seg_int64(rd_dtype, rd_op, int, bool) { return nullptr; }
SegFn seg_bits64(rd_op, int, bool) { return nullptr; }
SegFn seg_half(rd_dtype, rd_op, int, bool) { return nullptr; }
hipError_t rowreduce_fwd(const float*, int64_t, int64_t, rd_op, float*, void*, int, const Launch&, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t rowreduce_bwd(const float*, const float*, const void*, int64_t, int64_t, rd_op, float*, int,
                         const Launch&, hipStream_t, const SidePath&, unsigned*) {
  return hipErrorInvalidValue;
}
size_t rowreduce_saved_bytes(rd_op op, int64_t rows, int64_t cols) {
  // the same sizes as the real unit: 8 bytes per row for min/max; a 16-byte
  // header per row plus two doubles per 16,384-column chunk for product
  if (op == RD_MAX || op == RD_MIN) return (size_t)rows * 8;
  if (op == RD_PROD) return (size_t)rows * 16 + (size_t)rows * ((cols + 16383) / 16384) * 16;
  return 0;
}
hipError_t paper_design_reduce(const void*, int64_t, rd_dtype, int, int, void*, void*, int, int, hipStream_t) {
  return hipErrorInvalidValue;
}
}  // namespace rd
