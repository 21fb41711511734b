// eq_persist_queue.hpp -- the work queue of the persistent launch (EQ_F_PERSISTENT): how
// many items each queue step holds and which (stage, field, index) a queue position is.
// Host and device code, so that a host test checks the decode on every shape.
#pragma once

#include <hip/hip_runtime.h>

namespace eq {

struct PsArgs {
  int batch, nz;
  int gp, gt;               // planes per plane item, tiles per z item
  int nP, nZ;               // items per field of each plane stage, of the z stage
  int lag;                  // queue steps between a field's stages
  unsigned* ctr;            // [0] queue head, [1] workgroups done, [2] a bounded wait gave up,
                            // [4 + b] forward items done of field b, [4 + batch + b] z items done
  unsigned spin_limit;      // polls of a dependency before giving up (the kernel always ends)
};

// Items in queue steps 0 .. s-1.
__host__ __device__ inline int ps_prefix(const PsArgs& a, int s) {
  auto clampb = [&](int v) { return v < 0 ? 0 : (v > a.batch ? a.batch : v); };
  return a.nP * clampb(s) + a.nZ * clampb(s - a.lag) + a.nP * clampb(s - 2 * a.lag);
}

// Item q of the queue -> (stage 0 forward planes | 1 z tiles | 2 inverse planes, field, index):
// the step by bisection over the item counts, then forward, z and inverse items in that order.
__host__ __device__ inline void ps_decode(const PsArgs& a, int q, int& stage, int& b, int& j) {
  int lo = 0, hi = a.batch + 2 * a.lag;          // ps_prefix(lo) <= q < ps_prefix(hi)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ps_prefix(a, mid) <= q) lo = mid;
    else hi = mid;
  }
  int r = q - ps_prefix(a, lo);
  if (lo < a.batch) {
    if (r < a.nP) { stage = 0; b = lo; j = r; return; }
    r -= a.nP;
  }
  if (lo - a.lag >= 0 && lo - a.lag < a.batch) {
    if (r < a.nZ) { stage = 1; b = lo - a.lag; j = r; return; }
    r -= a.nZ;
  }
  stage = 2; b = lo - 2 * a.lag; j = r;
}

}  // namespace eq
