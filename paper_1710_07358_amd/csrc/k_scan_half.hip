// k_scan_half.hip -- instantiations of the scan kernels: float16 / bfloat16 and 16-bit bit patterns.
#include "scan.hpp"

namespace rd {

template <Store S, bool SEG> ScanFn scan_half_ops(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_SUM: return scan_pick<S, Op::Sum, SEG>(u, nt);
    case RD_PROD: return scan_pick<S, Op::Prod, SEG>(u, nt);
    case RD_MIN: return scan_pick<S, Op::Min, SEG>(u, nt);
    case RD_MAX: return scan_pick<S, Op::Max, SEG>(u, nt);
    case RD_AND: return scan_pick<Store::U16, Op::And, SEG>(u, nt);
    case RD_OR: return scan_pick<Store::U16, Op::Or, SEG>(u, nt);
    case RD_XOR: return scan_pick<Store::U16, Op::Xor, SEG>(u, nt);
  }
  return nullptr;
}

ScanFn scan_half(rd_dtype dt, rd_op op, bool seg, int u, bool nt) {
  if (dt == RD_F16) return seg ? scan_half_ops<Store::F16, true>(op, u, nt) : scan_half_ops<Store::F16, false>(op, u, nt);
  return seg ? scan_half_ops<Store::BF16, true>(op, u, nt) : scan_half_ops<Store::BF16, false>(op, u, nt);
}

}  // namespace rd
