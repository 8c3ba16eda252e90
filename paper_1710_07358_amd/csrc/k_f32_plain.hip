// k_f32_plain.hip -- instantiations of the plain and compensated kernels: float32 and its compensated sum.
#include "reduce_plain.hpp"

namespace rd {

PlainFn plain_f32(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_SUM: return pick<Red<Store::F32, Op::Sum>>(u, nt);
    case RD_PROD: return pick<Red<Store::F32, Op::Prod>>(u, nt);
    case RD_MIN: return pick<Red<Store::F32, Op::Min>>(u, nt);
    case RD_MAX: return pick<Red<Store::F32, Op::Max>>(u, nt);
    default: return plain_bits32(op, u, nt);
  }
}

PlainFn comp_f32(int u, bool nt) { return pick_comp<Store::F32>(u, nt); }

}  // namespace rd
