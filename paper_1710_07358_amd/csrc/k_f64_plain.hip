// k_f64_plain.hip -- instantiations of the plain and compensated kernels: float64 and 64-bit bit patterns.
#include "reduce_plain.hpp"

namespace rd {

PlainFn plain_f64(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_SUM: return pick<Red<Store::F64, Op::Sum>>(u, nt);
    case RD_PROD: return pick<Red<Store::F64, Op::Prod>>(u, nt);
    case RD_MIN: return pick<Red<Store::F64, Op::Min>>(u, nt);
    case RD_MAX: return pick<Red<Store::F64, Op::Max>>(u, nt);
    default: return plain_bits64(op, u, nt);
  }
}

}  // namespace rd
