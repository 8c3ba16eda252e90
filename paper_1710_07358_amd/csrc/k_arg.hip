// k_arg.hip -- instantiations of the arg-reduction kernel (min/max with the lowest index).
#include "reduce_arg.hpp"

namespace rd {

namespace {
template <Store S, bool MAX, bool NT> ArgFn arg_unroll(int u) {
  switch (u) {
    case 2: return launch_arg<S, MAX, 2, NT>;
    case 4: return launch_arg<S, MAX, 4, NT>;
    case 8: return launch_arg<S, MAX, 8, NT>;
  }
  return nullptr;
}
template <Store S> ArgFn arg_pick_fn(bool is_max, int u, bool nt) {
  if (is_max) return nt ? arg_unroll<S, true, true>(u) : arg_unroll<S, true, false>(u);
  return nt ? arg_unroll<S, false, true>(u) : arg_unroll<S, false, false>(u);
}
}  // namespace

ArgFn arg_launcher(rd_dtype dt, bool is_max, int unroll, bool nt) {
  switch (dt) {
    case RD_I32: return arg_pick_fn<Store::I32>(is_max, unroll, nt);
    case RD_U32: return arg_pick_fn<Store::U32>(is_max, unroll, nt);
    case RD_F32: return arg_pick_fn<Store::F32>(is_max, unroll, nt);
    case RD_F64: return arg_pick_fn<Store::F64>(is_max, unroll, nt);
    case RD_F16: return arg_pick_fn<Store::F16>(is_max, unroll, nt);
    case RD_BF16: return arg_pick_fn<Store::BF16>(is_max, unroll, nt);
    case RD_I64: return arg_pick_fn<Store::I64>(is_max, unroll, nt);
    case RD_U64: return arg_pick_fn<Store::U64>(is_max, unroll, nt);
  }
  return nullptr;
}

}  // namespace rd
