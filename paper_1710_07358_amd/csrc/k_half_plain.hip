// k_half_plain.hip -- instantiations of the plain and compensated kernels: float16 / bfloat16 (accumulated in float32) and 16-bit bit patterns.
#include "reduce_plain.hpp"

namespace rd {

template <Store S> PlainFn half_ops(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_SUM: return pick<Red<S, Op::Sum>>(u, nt);
    case RD_PROD: return pick<Red<S, Op::Prod>>(u, nt);
    case RD_MIN: return pick<Red<S, Op::Min>>(u, nt);
    case RD_MAX: return pick<Red<S, Op::Max>>(u, nt);
    case RD_AND: return pick<Red<Store::U16, Op::And>>(u, nt);
    case RD_OR: return pick<Red<Store::U16, Op::Or>>(u, nt);
    case RD_XOR: return pick<Red<Store::U16, Op::Xor>>(u, nt);
  }
  return nullptr;
}

PlainFn plain_half(rd_dtype dt, rd_op op, int u, bool nt) {
  return dt == RD_F16 ? half_ops<Store::F16>(op, u, nt) : half_ops<Store::BF16>(op, u, nt);
}

PlainFn comp_half(rd_dtype dt, int u, bool nt) {
  return dt == RD_F16 ? pick_comp<Store::F16>(u, nt) : pick_comp<Store::BF16>(u, nt);
}

}  // namespace rd
