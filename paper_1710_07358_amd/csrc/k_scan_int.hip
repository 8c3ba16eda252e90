// k_scan_int.hip -- instantiations of the scan kernels: int32 / uint32 and 32-bit bit patterns.
#include "scan.hpp"

namespace rd {

template <bool SEG> ScanFn scan_int_ops(rd_dtype dt, rd_op op, int u, bool nt) {
  const bool s = (dt == RD_I32);
  switch (op) {
    case RD_SUM: return scan_pick<Store::U32, Op::Sum, SEG>(u, nt);
    case RD_PROD: return scan_pick<Store::U32, Op::Prod, SEG>(u, nt);
    case RD_MIN: return s ? scan_pick<Store::I32, Op::Min, SEG>(u, nt) : scan_pick<Store::U32, Op::Min, SEG>(u, nt);
    case RD_MAX: return s ? scan_pick<Store::I32, Op::Max, SEG>(u, nt) : scan_pick<Store::U32, Op::Max, SEG>(u, nt);
    case RD_AND: return scan_pick<Store::U32, Op::And, SEG>(u, nt);
    case RD_OR: return scan_pick<Store::U32, Op::Or, SEG>(u, nt);
    case RD_XOR: return scan_pick<Store::U32, Op::Xor, SEG>(u, nt);
  }
  return nullptr;
}

// + and x wrap identically for int32 and uint32 (the unsigned code serves
// both); min/max compare by signedness.  and/or/xor of float32 data act on
// the same 32-bit patterns.
ScanFn scan_int(rd_dtype dt, rd_op op, bool seg, int u, bool nt) {
  return seg ? scan_int_ops<true>(dt, op, u, nt) : scan_int_ops<false>(dt, op, u, nt);
}

}  // namespace rd
