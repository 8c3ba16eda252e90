// k_half_seg.hip -- instantiations of the segmented kernels: float16 / bfloat16 and 16-bit bit patterns.
#include "reduce_segmented.hpp"

namespace rd {

template <Store S> SegFn half_seg_ops(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_SUM: return seg_pick<Red<S, Op::Sum>>(u, nt);
    case RD_PROD: return seg_pick<Red<S, Op::Prod>>(u, nt);
    case RD_MIN: return seg_pick<Red<S, Op::Min>>(u, nt);
    case RD_MAX: return seg_pick<Red<S, Op::Max>>(u, nt);
    case RD_AND: return seg_pick<Red<Store::U16, Op::And>>(u, nt);
    case RD_OR: return seg_pick<Red<Store::U16, Op::Or>>(u, nt);
    case RD_XOR: return seg_pick<Red<Store::U16, Op::Xor>>(u, nt);
  }
  return nullptr;
}

SegFn seg_half(rd_dtype dt, rd_op op, int u, bool nt) {
  return dt == RD_F16 ? half_seg_ops<Store::F16>(op, u, nt) : half_seg_ops<Store::BF16>(op, u, nt);
}

}  // namespace rd
