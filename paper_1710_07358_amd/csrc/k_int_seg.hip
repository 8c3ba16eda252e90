// k_int_seg.hip -- instantiations of the segmented kernels: int32 / uint32 and 32-bit bit patterns.
#include "reduce_segmented.hpp"

namespace rd {

SegFn seg_bits32(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_AND: return seg_pick<Red<Store::U32, Op::And>>(u, nt);
    case RD_OR: return seg_pick<Red<Store::U32, Op::Or>>(u, nt);
    case RD_XOR: return seg_pick<Red<Store::U32, Op::Xor>>(u, nt);
    default: return nullptr;
  }
}

SegFn seg_int(rd_dtype dt, rd_op op, int u, bool nt) {
  const bool s = (dt == RD_I32);
  switch (op) {
    case RD_SUM: return seg_pick<Red<Store::U32, Op::Sum>>(u, nt);
    case RD_PROD: return seg_pick<Red<Store::U32, Op::Prod>>(u, nt);
    case RD_MIN: return s ? seg_pick<Red<Store::I32, Op::Min>>(u, nt) : seg_pick<Red<Store::U32, Op::Min>>(u, nt);
    case RD_MAX: return s ? seg_pick<Red<Store::I32, Op::Max>>(u, nt) : seg_pick<Red<Store::U32, Op::Max>>(u, nt);
    default: return seg_bits32(op, u, nt);
  }
}

}  // namespace rd
