// k_scan_int64.hip -- instantiations of the scan kernels: int64 / uint64 and 64-bit bit patterns.
#include "scan.hpp"

namespace rd {

template <bool SEG> ScanFn scan_int64_ops(rd_dtype dt, rd_op op, int u, bool nt) {
  const bool s = (dt == RD_I64);
  switch (op) {
    case RD_SUM: return scan_pick<Store::U64, Op::Sum, SEG>(u, nt);
    case RD_PROD: return scan_pick<Store::U64, Op::Prod, SEG>(u, nt);
    case RD_MIN: return s ? scan_pick<Store::I64, Op::Min, SEG>(u, nt) : scan_pick<Store::U64, Op::Min, SEG>(u, nt);
    case RD_MAX: return s ? scan_pick<Store::I64, Op::Max, SEG>(u, nt) : scan_pick<Store::U64, Op::Max, SEG>(u, nt);
    case RD_AND: return scan_pick<Store::U64, Op::And, SEG>(u, nt);
    case RD_OR: return scan_pick<Store::U64, Op::Or, SEG>(u, nt);
    case RD_XOR: return scan_pick<Store::U64, Op::Xor, SEG>(u, nt);
  }
  return nullptr;
}

// and/or/xor of float64 data act on the same 64-bit patterns.
ScanFn scan_int64(rd_dtype dt, rd_op op, bool seg, int u, bool nt) {
  return seg ? scan_int64_ops<true>(dt, op, u, nt) : scan_int64_ops<false>(dt, op, u, nt);
}

}  // namespace rd
