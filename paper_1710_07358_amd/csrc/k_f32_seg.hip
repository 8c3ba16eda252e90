// k_f32_seg.hip -- instantiations of the segmented kernels: float32.
#include "reduce_segmented.hpp"

namespace rd {

SegFn seg_f32(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_SUM: return seg_pick<Red<Store::F32, Op::Sum>>(u, nt);
    case RD_PROD: return seg_pick<Red<Store::F32, Op::Prod>>(u, nt);
    case RD_MIN: return seg_pick<Red<Store::F32, Op::Min>>(u, nt);
    case RD_MAX: return seg_pick<Red<Store::F32, Op::Max>>(u, nt);
    default: return seg_bits32(op, u, nt);
  }
}

}  // namespace rd
