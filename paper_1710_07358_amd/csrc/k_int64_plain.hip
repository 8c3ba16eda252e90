// k_int64_plain.hip -- instantiations of the plain kernel: int64 / uint64 and 64-bit bit patterns.
#include "reduce_plain.hpp"

namespace rd {

PlainFn plain_bits64(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_AND: return pick<Red<Store::U64, Op::And>>(u, nt);
    case RD_OR: return pick<Red<Store::U64, Op::Or>>(u, nt);
    case RD_XOR: return pick<Red<Store::U64, Op::Xor>>(u, nt);
    default: return nullptr;
  }
}

// + and x wrap identically for int64 and uint64 (unsigned code); min/max differ.
PlainFn plain_int64(rd_dtype dt, rd_op op, int u, bool nt) {
  const bool s = (dt == RD_I64);
  switch (op) {
    case RD_SUM: return pick<Red<Store::U64, Op::Sum>>(u, nt);
    case RD_PROD: return pick<Red<Store::U64, Op::Prod>>(u, nt);
    case RD_MIN: return s ? pick<Red<Store::I64, Op::Min>>(u, nt) : pick<Red<Store::U64, Op::Min>>(u, nt);
    case RD_MAX: return s ? pick<Red<Store::I64, Op::Max>>(u, nt) : pick<Red<Store::U64, Op::Max>>(u, nt);
    default: return plain_bits64(op, u, nt);
  }
}

}  // namespace rd
