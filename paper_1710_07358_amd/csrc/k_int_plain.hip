// k_int_plain.hip -- instantiations of the plain and compensated kernels: int32 / uint32 and 32-bit bit patterns.
#include "reduce_plain.hpp"

namespace rd {

PlainFn plain_bits32(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_AND: return pick<Red<Store::U32, Op::And>>(u, nt);
    case RD_OR: return pick<Red<Store::U32, Op::Or>>(u, nt);
    case RD_XOR: return pick<Red<Store::U32, Op::Xor>>(u, nt);
    default: return nullptr;
  }
}

// Integer + and x wrap identically for int32 and uint32, so both use the
// unsigned code; only min/max compare differently.
PlainFn plain_int(rd_dtype dt, rd_op op, int u, bool nt) {
  const bool s = (dt == RD_I32);
  switch (op) {
    case RD_SUM: return pick<Red<Store::U32, Op::Sum>>(u, nt);
    case RD_PROD: return pick<Red<Store::U32, Op::Prod>>(u, nt);
    case RD_MIN: return s ? pick<Red<Store::I32, Op::Min>>(u, nt) : pick<Red<Store::U32, Op::Min>>(u, nt);
    case RD_MAX: return s ? pick<Red<Store::I32, Op::Max>>(u, nt) : pick<Red<Store::U32, Op::Max>>(u, nt);
    default: return plain_bits32(op, u, nt);
  }
}

}  // namespace rd
