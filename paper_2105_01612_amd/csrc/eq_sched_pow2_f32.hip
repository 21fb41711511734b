// Compile-time radix schedules, powers of two, FP32 (see eq_sched.hpp).
#include "eq_sched.hpp"

namespace eq {
template <> bool ct_launch_pow2<float>(const FastArgs<float>& a) { return ct_launch_pow2_impl<float>(a); }
}  // namespace eq
