// k_scan_f64.hip -- instantiations of the scan kernels: float64.
#include "scan.hpp"

namespace rd {

template <bool SEG> ScanFn scan_f64_ops(rd_op op, int u, bool nt) {
  switch (op) {
    case RD_SUM: return scan_pick<Store::F64, Op::Sum, SEG>(u, nt);
    case RD_PROD: return scan_pick<Store::F64, Op::Prod, SEG>(u, nt);
    case RD_MIN: return scan_pick<Store::F64, Op::Min, SEG>(u, nt);
    case RD_MAX: return scan_pick<Store::F64, Op::Max, SEG>(u, nt);
    default: return nullptr;  // bitwise: the 64-bit pattern kernels
  }
}

ScanFn scan_f64(rd_op op, bool seg, int u, bool nt) { return seg ? scan_f64_ops<true>(op, u, nt) : scan_f64_ops<false>(op, u, nt); }

}  // namespace rd
