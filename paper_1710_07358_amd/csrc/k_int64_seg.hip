// k_int64_seg.hip -- instantiations of the segmented kernel: int64 / uint64 and 64-bit bit patterns.
#include "reduce_segmented.hpp"

namespace rd {

SegFn seg_bits64(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_AND: return seg_pick<Red<Store::U64, Op::And>>(u, nt);
    case RD_OR: return seg_pick<Red<Store::U64, Op::Or>>(u, nt);
    case RD_XOR: return seg_pick<Red<Store::U64, Op::Xor>>(u, nt);
    default: return nullptr;
  }
}

SegFn seg_int64(rd_dtype dt, rd_op op, int u, bool nt) {
  const bool s = (dt == RD_I64);
  switch (op) {
    case RD_SUM: return seg_pick<Red<Store::U64, Op::Sum>>(u, nt);
    case RD_PROD: return seg_pick<Red<Store::U64, Op::Prod>>(u, nt);
    case RD_MIN: return s ? seg_pick<Red<Store::I64, Op::Min>>(u, nt) : seg_pick<Red<Store::U64, Op::Min>>(u, nt);
    case RD_MAX: return s ? seg_pick<Red<Store::I64, Op::Max>>(u, nt) : seg_pick<Red<Store::U64, Op::Max>>(u, nt);
    default: return seg_bits64(op, u, nt);
  }
}

}  // namespace rd
