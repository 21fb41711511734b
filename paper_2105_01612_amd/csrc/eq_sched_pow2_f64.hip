// Compile-time radix schedules, powers of two, FP64 (see eq_sched.hpp).
#include "eq_sched.hpp"

namespace eq {
template <> bool ct_launch_pow2<double>(const FastArgs<double>& a) { return ct_launch_pow2_impl<double>(a); }
}  // namespace eq
