// Compile-time radix schedules with a factor 3 or 5, FP32 and FP64 (see eq_sched.hpp).
#include "eq_sched.hpp"

namespace eq {
template <> bool ct_launch_mixed<float>(const FastArgs<float>& a) { return ct_launch_mixed_impl<float>(a); }
template <> bool ct_launch_mixed<double>(const FastArgs<double>& a) { return ct_launch_mixed_impl<double>(a); }
}  // namespace eq
