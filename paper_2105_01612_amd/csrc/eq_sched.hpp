// eq_sched.hpp -- compile-time radix schedules for the common grid edges.  Each
// schedule mirrors what the planner picks for that (n, E) (factor_axis in
// eq_capi.cpp); a launch is taken here only when the run-time radix list matches.
#pragma once

#include "eq_kernels_impl.hpp"

namespace eq {

template <int... Rs>
bool radices_match(const FftDesc& d) {
  constexpr int rs[] = {Rs...};
  if (d.nst != (int)sizeof...(Rs)) return false;
  for (int i = 0; i < d.nst; ++i)
    if (d.r[i] != rs[i]) return false;
  return true;
}

template <typename T, int... Rs>
bool try_sched(const FastArgs<T>& a) {
  using S = Sched<Rs...>;
  if (a.n != S::N || a.E != S::E || !radices_match<Rs...>(a.d)) return false;
  if (a.kind == KK_X6S && !(S::N / S::E <= 32 || S::N / S::E == 64)) return false;
  if (!a.dry) launch_with<T, S>(a);
  return true;
}

// radix 4 (E = 4): only the six-component x kernel takes it (FP32; its 6 * E values per lane)
template <typename T, int... Rs>
bool try_sched_x6(const FastArgs<T>& a) {
  using S = Sched<Rs...>;
  if (a.n != S::N || a.E != S::E || !radices_match<Rs...>(a.d)) return false;
  if (a.kind == KK_X6) {
    if (!a.dry) hipLaunchKernelGGL((k_x6_r<T, S>), a.grid, a.block, a.lds, a.s, a.W, a.xa, a.d, a.tw, a.sym);
    return true;
  }
  if (a.kind == KK_X6S) {
    if constexpr (S::N / S::E <= 32) {
      if (!a.dry) hipLaunchKernelGGL((k_x6s_r<T, S>), a.grid, a.block, a.lds, a.s, a.W, a.xa, a.d, a.tw, a.sym);
      return true;
    } else if constexpr (S::N / S::E == 64) {
      if (!a.dry) hipLaunchKernelGGL((k_x6w_r<T, S>), a.grid, a.block, a.lds, a.s, a.W, a.xa, a.d, a.tw, a.sym);
      return true;
    }
  }
  return false;
}

// radix 4 with a factor 3 or 5 (E = 12, 20): only the split six-component x kernel takes it
template <typename T, int... Rs>
bool try_sched_x6s(const FastArgs<T>& a) {
  using S = Sched<Rs...>;
  if (a.n != S::N || a.E != S::E || !radices_match<Rs...>(a.d) || a.kind != KK_X6S) return false;
  static_assert(S::N / S::E <= 32, "the split kernel needs nx / E to divide 32");
  if (!a.dry) hipLaunchKernelGGL((k_x6s_r<T, S>), a.grid, a.block, a.lds, a.s, a.W, a.xa, a.d, a.tw, a.sym);
  return true;
}

// powers of two: radix 8 (E = 8) and radix 16 (E = 16)
template <typename T>
bool ct_launch_pow2_impl(const FastArgs<T>& a) {
  if (a.E == 4) {
    if constexpr (sizeof(T) == 4)
      return try_sched_x6<T, 4, 4, 2>(a) || try_sched_x6<T, 4, 4, 4>(a) || try_sched_x6<T, 4, 4, 4, 2>(a) ||
             try_sched_x6<T, 4, 4, 4, 4>(a) || try_sched_x6<T, 4, 4, 4, 4, 2>(a);
    return false;
  }
  return try_sched<T, 8, 4>(a) || try_sched<T, 8, 8>(a) || try_sched<T, 8, 8, 2>(a) || try_sched<T, 8, 8, 4>(a) ||
         try_sched<T, 8, 8, 8>(a) || try_sched<T, 16, 8>(a) || try_sched<T, 16, 16>(a) || try_sched<T, 16, 16, 2>(a);
}

// a factor 3 (E = 24) or 5 (E = 40); radix-4 schedules with a factor 3 (E = 12) or 5 (E = 20)
// for the split six-component x kernel only (FP32)
template <typename T>
bool ct_launch_mixed_impl(const FastArgs<T>& a) {
  if (a.E == 12 || a.E == 20) {
    if constexpr (sizeof(T) == 4)
      return try_sched_x6s<T, 4, 4, 2, 3>(a) || try_sched_x6s<T, 4, 4, 4, 3>(a) || try_sched_x6s<T, 4, 4, 4, 2, 3>(a) ||
             try_sched_x6s<T, 4, 4, 2, 5>(a) || try_sched_x6s<T, 4, 4, 4, 5>(a);
    return false;
  }
  return try_sched<T, 8, 4, 3>(a) || try_sched<T, 8, 8, 3>(a) || try_sched<T, 8, 8, 2, 3>(a) ||
         try_sched<T, 8, 4, 5>(a);
}

}  // namespace eq
