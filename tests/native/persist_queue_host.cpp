// Host check of the persistent launch's work queue (eq_persist_queue.hpp): for many batch
// sizes, item counts and lags, queue positions 0 .. total-1 decode to every (stage, field,
// index) exactly once, and every item that waits (a z item on its field's forward items, an
// inverse item on its field's z items) comes after all the items it waits for, so a waiter
// only ever waits on items claimed before it.  Prints "ok <cases>" or the first failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "eq_persist_queue.hpp"

using namespace eq;

static int check(int batch, int nP, int nZ, int lag) {
  PsArgs a{};
  a.batch = batch; a.nP = nP; a.nZ = nZ; a.lag = lag;
  const int total = batch * (2 * nP + nZ);
  if (ps_prefix(a, batch + 2 * lag) != total) return 1;
  // position of every item: pos[stage][field][index]
  std::vector<int> fwd((size_t)batch * nP, -1), zz((size_t)batch * nZ, -1), inv((size_t)batch * nP, -1);
  for (int q = 0; q < total; ++q) {
    int st = -1, b = -1, j = -1;
    ps_decode(a, q, st, b, j);
    if (b < 0 || b >= batch || j < 0) return 2;
    std::vector<int>& v = st == 0 ? fwd : st == 1 ? zz : inv;
    const int n = st == 1 ? nZ : nP;
    if (st < 0 || st > 2 || j >= n) return 3;
    int& slot = v[(size_t)b * n + j];
    if (slot != -1) return 4;                   // decoded twice
    slot = q;
  }
  for (int b = 0; b < batch; ++b) {
    int last_f = -1, first_z = total, last_z = -1, first_i = total;
    for (int j = 0; j < nP; ++j) {
      if (fwd[(size_t)b * nP + j] < 0 || inv[(size_t)b * nP + j] < 0) return 5;
      last_f = fwd[(size_t)b * nP + j] > last_f ? fwd[(size_t)b * nP + j] : last_f;
      first_i = inv[(size_t)b * nP + j] < first_i ? inv[(size_t)b * nP + j] : first_i;
    }
    for (int j = 0; j < nZ; ++j) {
      const int p = zz[(size_t)b * nZ + j];
      if (p < 0) return 5;
      first_z = p < first_z ? p : first_z;
      last_z = p > last_z ? p : last_z;
    }
    if (!(last_f < first_z && last_z < first_i)) return 6;   // a waiter before what it waits for
  }
  return 0;
}

int main() {
  int cases = 0;
  const int batches[] = {1, 2, 3, 5, 8, 9, 17, 64, 100};
  const int nps[] = {1, 2, 24, 96, 384, 768};
  const int nzs[] = {1, 3, 33, 132, 264};
  for (int batch : batches)
    for (int nP : nps)
      for (int nZ : nzs)
        for (int lag = 1; lag <= 12; lag += (lag < 4 ? 1 : 4)) {
          const int e = check(batch, nP, nZ, lag);
          ++cases;
          if (e) {
            std::printf("FAIL %d: batch %d nP %d nZ %d lag %d\n", e, batch, nP, nZ, lag);
            return 1;
          }
        }
  std::printf("ok %d\n", cases);
  return 0;
}
