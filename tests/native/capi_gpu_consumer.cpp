// A program that uses libeq through include/eq.h alone: device buffers from hipMalloc, the
// null stream, no Python and no torch.  It checks properties that hold by definition of the
// projection (Section 3.2) and need none of its arithmetic here:
//   - a plane wave A cos(2 pi k x / N) along x plus a constant keeps the constant and the
//     components 22, 33, 23 of A and loses 11, 12, 13 (the normal of every nonzero
//     frequency it holds is the x axis, for both operators);
//   - the output's divergence residual is at round-off (eq_residual);
//   - projecting the output again changes nothing (idempotence);
//   - output + removed part = input;
//   - an edge with a prime factor 7 is refused with EQ_ERR_SIZE before any device work.
// Exit status 0 when every check passes; each check prints one line.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "eq.h"

namespace {

int failures = 0;

void check(bool ok, const char* what, double value, double bound) {
  std::printf("%s %s: %.3e (bound %.1e)\n", ok ? "PASS" : "FAIL", what, value, bound);
  if (!ok) ++failures;
}

bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  std::printf("FAIL %s: %s\n", what, hipGetErrorString(e));
  ++failures;
  return false;
}

bool eq_ok(eq_status s, const char* what) {
  if (s == EQ_OK) return true;
  std::printf("FAIL %s: %s (%s)\n", what, eq_status_str(s), eq_last_error());
  ++failures;
  return false;
}

void run(int op, const char* name) {
  const int n = 32, k = 3;
  const size_t M = (size_t)n * n * n;
  // Voigt order 11, 22, 33, 23, 13, 12; weights 2 on the off-diagonals for the Frobenius norm
  const double A[6] = {1.0, 2.0, -3.0, 0.5, -0.7, 1.3}, c0[6] = {10.0, -4.0, 7.0, 2.0, -1.0, 3.0};
  const bool kept[6] = {false, true, true, true, false, false};
  std::vector<double> S(6 * M), want(6 * M);
  for (int c = 0; c < 6; ++c)
    for (size_t e = 0; e < M; ++e) {
      const int x = (int)(e % n);
      const double w = std::cos(2.0 * M_PI * k * x / n);
      S[c * M + e] = c0[c] + A[c] * w;
      want[c * M + e] = c0[c] + (kept[c] ? A[c] * w : 0.0);
    }
  eq_desc d{};
  d.nx = d.ny = d.nz = n;
  d.batch = 1;
  d.op = op;
  d.prec = EQ_FP64;
  d.h = 1.0;
  d.flags = 0;
  eq_plan_t p = nullptr;
  if (!eq_ok(eq_plan(&d, nullptr, &p), "eq_plan")) return;
  double *dS = nullptr, *dOut = nullptr, *dRem = nullptr, *dOut2 = nullptr;
  const size_t bytes = 6 * M * sizeof(double);
  if (hip_ok(hipMalloc((void**)&dS, bytes), "hipMalloc") && hip_ok(hipMalloc((void**)&dOut, bytes), "hipMalloc") &&
      hip_ok(hipMalloc((void**)&dRem, bytes), "hipMalloc") && hip_ok(hipMalloc((void**)&dOut2, bytes), "hipMalloc") &&
      hip_ok(hipMemcpy(dS, S.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy") &&
      eq_ok(eq_project(p, dS, dOut, dRem), "eq_project") && eq_ok(eq_project(p, dOut, dOut2, nullptr), "eq_project") &&
      hip_ok(hipDeviceSynchronize(), "hipDeviceSynchronize")) {
    std::vector<double> out(6 * M), rem(6 * M), out2(6 * M);
    hip_ok(hipMemcpy(out.data(), dOut, bytes, hipMemcpyDeviceToHost), "hipMemcpy");
    hip_ok(hipMemcpy(rem.data(), dRem, bytes, hipMemcpyDeviceToHost), "hipMemcpy");
    hip_ok(hipMemcpy(out2.data(), dOut2, bytes, hipMemcpyDeviceToHost), "hipMemcpy");
    double e_want = 0.0, e_sum = 0.0, e_idem = 0.0;
    for (size_t i = 0; i < 6 * M; ++i) {
      e_want = std::fmax(e_want, std::fabs(out[i] - want[i]));
      e_sum = std::fmax(e_sum, std::fabs(out[i] + rem[i] - S[i]));
      e_idem = std::fmax(e_idem, std::fabs(out2[i] - out[i]));
    }
    char what[96];
    std::snprintf(what, sizeof what, "%s plane wave: max |out - closed form| (MPa)", name);
    check(e_want <= 1e-12, what, e_want, 1e-12);
    std::snprintf(what, sizeof what, "%s out + removed = in: max abs", name);
    check(e_sum <= 1e-12, what, e_sum, 1e-12);
    std::snprintf(what, sizeof what, "%s idempotence: max |P(P(S)) - P(S)|", name);
    check(e_idem <= 1e-12, what, e_idem, 1e-12);
    double norms[3] = {0.0, 0.0, 0.0};
    if (eq_ok(eq_residual(p, dOut, norms, nullptr), "eq_residual")) {
      std::snprintf(what, sizeof what, "%s residual of the output, rel", name);
      check(norms[2] <= 1e-13, what, norms[2], 1e-13);
    }
    if (eq_ok(eq_residual(p, dS, norms, nullptr), "eq_residual")) {
      std::snprintf(what, sizeof what, "%s residual of the input, rel (not equilibrated)", name);
      check(norms[2] > 1e-3, what, norms[2], 1e-3);
    }
  }
  hipFree(dS);
  hipFree(dOut);
  hipFree(dRem);
  hipFree(dOut2);
  eq_ok(eq_plan_destroy(p), "eq_plan_destroy");
}

}  // namespace

int main() {
  std::printf("%s\n", eq_version());
  run(EQ_OP_DDO, "DDO");
  run(EQ_OP_CDO, "CDO");
  eq_desc bad{};
  bad.nx = 14;                  // 2 * 7: a prime factor outside {2, 3, 5}
  bad.ny = bad.nz = 16;
  bad.batch = 1;
  bad.op = EQ_OP_DDO;
  bad.prec = EQ_FP64;
  bad.h = 1.0;
  eq_plan_t p = nullptr;
  const eq_status s = eq_plan(&bad, nullptr, &p);
  check(s == EQ_ERR_SIZE && p == nullptr, "nx = 14 refused with EQ_ERR_SIZE (status)", (double)s, (double)EQ_ERR_SIZE);
  std::printf("%s\n", failures ? "FAILED" : "ALL PASSED");
  return failures ? 1 : 0;
}
