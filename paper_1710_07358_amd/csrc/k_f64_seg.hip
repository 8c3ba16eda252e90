// k_f64_seg.hip -- instantiations of the segmented kernels: float64 and 64-bit bit patterns.
#include "reduce_segmented.hpp"

namespace rd {

SegFn seg_f64(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_SUM: return seg_pick<Red<Store::F64, Op::Sum>>(u, nt);
    case RD_PROD: return seg_pick<Red<Store::F64, Op::Prod>>(u, nt);
    case RD_MIN: return seg_pick<Red<Store::F64, Op::Min>>(u, nt);
    case RD_MAX: return seg_pick<Red<Store::F64, Op::Max>>(u, nt);
    default: return seg_bits64(op, u, nt);
  }
}

}  // namespace rd
