// Host-side logic of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer:
// grid validation, radix factorization, workspace layout, the EQ_TUNE parser, the
// status strings and the plan's failure path without a device.  The translation unit
// includes eq_capi.cpp itself, so the functions of its anonymous namespace are
// reachable; the kernel translation units are linked host-only (no kernel is launched).
// Prints "ok <checks>" and exits 0, or names the first failed check and exits 1.
#include "eq_capi.cpp"

#include <cstdio>
#include <cstdlib>
#include <string>

namespace {

int g_checks = 0;

#define CHECK(cond, ...)                                  \
  do {                                                    \
    ++g_checks;                                           \
    if (!(cond)) {                                        \
      std::fprintf(stderr, "FAILED %s: ", #cond);         \
      std::fprintf(stderr, __VA_ARGS__);                  \
      std::fprintf(stderr, "\n");                         \
      std::exit(1);                                       \
    }                                                     \
  } while (0)

bool smooth_even(int n) {
  if (n < 4 || n > 1024 || (n & 1)) return false;
  int m = n;
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  return m == 1;
}

void check_factor_axis() {
  for (int n = -3; n <= 1100; ++n) {
    for (int mode = 0; mode < 3; ++mode) {
      AxisFft a{};
      const bool ok = factor_axis(n, &a, mode == 1, mode == 2);
      CHECK(ok == smooth_even(n), "n=%d mode=%d ok=%d", n, mode, (int)ok);
      if (!ok) continue;
      long prod = 1;
      CHECK(a.d.nst >= 1 && a.d.nst <= kMaxStages, "n=%d nst=%d", n, a.d.nst);
      for (int s = 0; s < a.d.nst; ++s) {
        const int r = a.d.r[s];
        CHECK(r == 2 || r == 3 || r == 4 || r == 5 || r == 8 || r == 16, "n=%d radix %d", n, r);
        if (a.fast) CHECK(a.E % r == 0, "n=%d E=%d radix %d", n, a.E, r);
        prod *= r;
      }
      CHECK(prod == n && a.d.n == n, "n=%d product %ld", n, prod);
      CHECK(n % a.E == 0, "n=%d E=%d", n, a.E);
    }
  }
}

eq_desc desc(int nx, int ny, int nz, int batch = 1, int op = EQ_OP_DDO, int prec = EQ_FP32, double h = 1.0,
             unsigned flags = 0) {
  eq_desc d{};
  d.nx = nx; d.ny = ny; d.nz = nz; d.batch = batch; d.op = op; d.prec = prec; d.h = h; d.flags = flags;
  return d;
}

void check_validate_and_layout() {
  CHECK(validate(nullptr) == EQ_ERR_ARG, "null");
  eq_desc d = desc(32, 32, 32, 0);
  CHECK(validate(&d) == EQ_ERR_ARG, "batch 0");
  d = desc(32, 32, 32, 1, 7);
  CHECK(validate(&d) == EQ_ERR_ARG, "op");
  d = desc(32, 32, 32, 1, EQ_OP_CDO, 9);
  CHECK(validate(&d) == EQ_ERR_ARG, "prec");
  for (double h : {0.0, -1.0, HUGE_VAL, std::nan("")}) {
    d = desc(32, 32, 32, 1, EQ_OP_DDO, EQ_FP64, h);
    CHECK(validate(&d) == EQ_ERR_ARG, "h=%g", h);
  }
  d = desc(32, 32, 32, 1, EQ_OP_DDO, EQ_FP64, 1.0, EQ_F_PERSISTENT << 8);
  CHECK(validate(&d) == EQ_ERR_ARG, "unknown flag");
  for (int n : {0, 2, 3, 7, 14, 1026, 2048, 98})
    for (int axis = 0; axis < 3; ++axis) {
      int e[3] = {32, 32, 32};
      e[axis] = n;
      d = desc(e[0], e[1], e[2]);
      CHECK(validate(&d) == EQ_ERR_SIZE, "edge %d on axis %d", n, axis);
      size_t bytes = 0;
      CHECK(eq_plan_footprint(&d, &bytes) == EQ_ERR_SIZE, "footprint edge %d", n);
      CHECK(std::strlen(eq_last_error()) > 0, "message");
    }
  // batch so large that the launch grids overflow
  d = desc(1024, 1024, 1024, 4000);
  CHECK(validate(&d) == EQ_ERR_SIZE, "rows");
  size_t bytes = 0;
  CHECK(eq_plan_footprint(&d, nullptr) == EQ_ERR_ARG, "null bytes");
  // every accepted edge: the footprint covers the workspace and the tables
  for (int n = 4; n <= 1024; n += 2) {
    if (!smooth_even(n)) continue;
    for (int prec : {EQ_FP32, EQ_FP64}) {
      d = desc(n, 4, 6, 2, EQ_OP_CDO, prec);
      const eq_status st = eq_plan_footprint(&d, &bytes);
      CHECK(st == EQ_OK || st == EQ_ERR_SIZE, "n=%d status %d", n, (int)st);
      if (st != EQ_OK) continue;
      const size_t es = prec == EQ_FP64 ? 8 : 4;
      const Layout L = layout_of(&d);
      CHECK(bytes == L.total(), "n=%d", n);
      CHECK(L.w_bytes >= (size_t)2 * 6 * (6 / 2 + 1) * 4 * n * 2 * es, "n=%d workspace", n);
      CHECK(L.tw32_bytes == (size_t)(n + 4 + 6) * sizeof(float2), "n=%d twiddles", n);
    }
  }
  // the three-pass spectrum (half along x) never exceeds the workspace
  for (int n : {64, 128, 256})
    for (int nz : {64, 128, 256}) {
      d = desc(n, n, nz, 3);
      const Layout L = layout_of(&d);
      CHECK(L.w_bytes >= (size_t)3 * 6 * nz * n * (n / 2 + 1) * 2 * 4, "three-pass %d %d", n, nz);
    }
}

void check_symbol_max() {
  for (int op : {EQ_OP_CDO, EQ_OP_DDO})
    for (int n : {4, 6, 8, 96, 256}) {
      eq_desc d = desc(n, 2 * n, 6, 1, op, EQ_FP64, 0.5);
      double direct = 0.0;
      const int dims[3] = {n, 2 * n, 6};
      double m[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a)
        for (int q = 0; q < dims[a]; ++q) {
          double s;
          if (op == EQ_OP_CDO) {
            const int k = 2 * q < dims[a] ? q : (2 * q == dims[a] ? 0 : q - dims[a]);
            s = 2.0 * M_PI * k / (dims[a] * 0.5);
          } else {
            s = (2 * q) % dims[a] == 0 ? 0.0 : std::sin(2.0 * M_PI * q / dims[a]) / 0.5;
          }
          m[a] = std::max(m[a], s * s);
        }
      direct = m[0] + m[1] + m[2];
      CHECK(std::fabs(symbol_max2(&d) - direct) <= 1e-12 * direct, "op=%d n=%d", op, n);
    }
}

void check_tune_parser() {
  const struct { const char* env; int tx_y, tx_z, rw_x, chunk, radix16, schedule, tc_zp, radix4, xsplit, zp_e; } cases[] = {
      {"tx_y=16,tx_z=32,rw_x=4,chunk=32,radix16=2,schedule=5", 16, 32, 4, 32, 2, 5, 0, 0, 0, 0},
      {"schedule=3 tc_zp=8", 0, 0, 0, 0, -1, 3, 8, 0, 0, 0},
      {"zp_e=4,schedule=3", 0, 0, 0, 0, -1, 3, 0, 0, 0, 4},
      {"radix4=1,xsplit=2,,", 0, 0, 0, 0, -1, 0, 0, 1, 2, 0},
      {"", 0, 0, 0, 0, -1, 0, 0, 0, 0, 0},
      {",,,=,=5,tx_y=,unknown=3,tx_z", 0, 0, 0, 0, -1, 0, 0, 0, 0, 0},
      {"tx_y=abc,rw_x=-3", 0, 0, -3, 0, -1, 0, 0, 0, 0, 0},
  };
  for (const auto& c : cases) {
    setenv("EQ_TUNE", c.env, 1);
    const Tune t = tune_from_env();
    CHECK(t.tx_y == c.tx_y && t.tx_z == c.tx_z && t.rw_x == c.rw_x && t.chunk == c.chunk && t.radix16 == c.radix16 &&
              t.schedule == c.schedule && t.tc_zp == c.tc_zp && t.radix4 == c.radix4 && t.xsplit == c.xsplit &&
              t.zp_e == c.zp_e,
          "EQ_TUNE=\"%s\"", c.env);
  }
  std::string longv;
  for (int i = 0; i < 2000; ++i) longv += "tx_y=8,";
  setenv("EQ_TUNE", longv.c_str(), 1);
  CHECK(tune_from_env().tx_y == 8, "long");
  unsetenv("EQ_TUNE");
  const Tune t = tune_from_env();
  CHECK(t.tx_y == 0 && t.radix16 == -1, "unset");
}

void check_status_strings() {
  for (int s = 0; s < 8; ++s) {          // every value the enumeration can hold in C++
    const char* str = eq_status_str((eq_status)s);
    CHECK(str && std::strncmp(str, "EQ_", 3) == 0, "status %d", s);
  }
  CHECK(std::strcmp(eq_status_str(EQ_ERR_NONFINITE), "EQ_ERR_NONFINITE") == 0, "nonfinite");
  CHECK(std::strncmp(eq_version(), "libeq", 5) == 0, "version");
}

void check_ranges_overlap() {
  // a div_out of three components ending where the six-component field begins does not
  // overlap it (each range is taken with its own length)
  alignas(16) static unsigned char buf[4096];
  const size_t F = 64;                                 // bytes of one component of the batch
  unsigned char* field = buf + 3 * F;
  CHECK(!ranges_overlap(buf, 3 * F, field, 6 * F), "adjacent below");
  CHECK(ranges_overlap(buf + 1, 3 * F, field, 6 * F), "one byte into the field");
  CHECK(!ranges_overlap(field + 6 * F, 3 * F, field, 6 * F), "adjacent above");
  CHECK(ranges_overlap(field + 6 * F - 1, 3 * F, field, 6 * F), "last byte of the field");
  CHECK(ranges_overlap(field + F, 3 * F, field, 6 * F), "inside");
  CHECK(ranges_overlap(field, 6 * F, field, 6 * F), "same range");
}

void check_plan_without_device() {
  // null arguments are refused before any device call
  eq_plan_t p = reinterpret_cast<eq_plan_t>(0x1);
  CHECK(eq_plan(nullptr, nullptr, &p) == EQ_ERR_ARG && p == nullptr, "null desc");
  eq_desc d = desc(16, 16, 16);
  CHECK(eq_plan(&d, nullptr, nullptr) == EQ_ERR_ARG, "null out");
  CHECK(eq_project(nullptr, nullptr, nullptr, nullptr) == EQ_ERR_ARG, "project null plan");
  CHECK(eq_residual(nullptr, nullptr, nullptr, nullptr) == EQ_ERR_ARG, "residual null plan");
  CHECK(eq_plan_destroy(nullptr) == EQ_ERR_ARG, "destroy null");
  CHECK(eq_plan_tune(nullptr, nullptr) == EQ_ERR_ARG, "tune null");
  // with no device visible the plan fails cleanly (its partial state is released)
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    const eq_status st = eq_plan(&d, nullptr, &p);
    CHECK(st == EQ_ERR_DEVICE && p == nullptr, "no device: status %d", (int)st);
  }
}

}  // namespace

int main() {
  check_factor_axis();
  check_validate_and_layout();
  check_symbol_max();
  check_tune_parser();
  check_status_strings();
  check_ranges_overlap();
  check_plan_without_device();
  std::printf("ok %d\n", g_checks);
  return 0;
}
