// k_scan_int.hip -- instantiations of the scan kernels: int32 / uint32 and 32-bit bit patterns.
#include "scan.hpp"

namespace rd {

template <bool SEG> ScanFn scan_int_ops(rd_dtype dt, rd_op op, bool nt) {
  const bool s = (dt == RD_I32);
  switch (op) {
    case RD_SUM: return scan_pick<Store::U32, Op::Sum, SEG>(nt);
    case RD_PROD: return scan_pick<Store::U32, Op::Prod, SEG>(nt);
    case RD_MIN: return s ? scan_pick<Store::I32, Op::Min, SEG>(nt) : scan_pick<Store::U32, Op::Min, SEG>(nt);
    case RD_MAX: return s ? scan_pick<Store::I32, Op::Max, SEG>(nt) : scan_pick<Store::U32, Op::Max, SEG>(nt);
    case RD_AND: return scan_pick<Store::U32, Op::And, SEG>(nt);
    case RD_OR: return scan_pick<Store::U32, Op::Or, SEG>(nt);
    case RD_XOR: return scan_pick<Store::U32, Op::Xor, SEG>(nt);
  }
  return nullptr;
}

// + and x wrap identically for int32 and uint32 (the unsigned code serves
// both); min/max compare by signedness.  and/or/xor of float32 data act on
// the same 32-bit patterns.
ScanFn scan_int(rd_dtype dt, rd_op op, bool seg, bool nt) {
  return seg ? scan_int_ops<true>(dt, op, nt) : scan_int_ops<false>(dt, op, nt);
}

}  // namespace rd
