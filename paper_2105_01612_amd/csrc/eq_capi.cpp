// eq_capi.cpp -- plan object and C ABI of libeq (declared in include/eq.h).
//
// Host-side responsibilities: argument validation before any device work,
// radix schedules per axis, device workspace and FP64 tables, stream binding,
// the pass sequence of eq_project / eq_residual, optional hipGraph replay,
// per-pass event timing, and status codes (nothing aborts or throws across
// the ABI).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "eq.h"
#include "eq_internal.hpp"

using namespace eq;

namespace {

thread_local std::string g_last_error;

eq_status fail(eq_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

eq_status hip_fail(hipError_t e, const char* what) {
  return fail(EQ_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define EQ_HIP(call, what)                         \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool fault_inject_alloc() {
  const char* v = std::getenv("EQ_FAULT_INJECT");
  return v && std::strcmp(v, "alloc") == 0;
}

// Radix schedules.  Register engine (every radix divides E): powers of two use 8s
// (E = 8) or, with `wide` and n >= 128, 16s (E = 16), with one 2/4/8 to finish; a factor 3 or 5
// switches to E = 24 or 40 with the power of two in 8s and 4/2.  Edges with both
// 3 and 5, or fewer than three factors of 2, use the generic engine.
bool factor_axis(int n, AxisFft* out, bool wide = false, bool narrow = false) {
  if (n < 4 || n > 1024 || (n & 1)) return false;
  int m = n, a = 0, b = 0, c = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  while (m % 5 == 0) { m /= 5; ++c; }
  if (m != 1) return false;
  FftDesc d{};
  d.n = n;
  int k = 0;
  if (narrow && a >= 3 && !(b > 0 && c > 0)) {
    // radix-4 stages (E = 4; with a factor 3 or 5, E = 12 or 20): a third to a half of the
    // registers per lane of the radix-8 schedules
    for (int i = 0; i < a / 2; ++i) d.r[k++] = 4;
    if (a % 2) d.r[k++] = 2;
    for (int i = 0; i < b; ++i) d.r[k++] = 3;
    for (int i = 0; i < c; ++i) d.r[k++] = 5;
    if (k > kMaxStages) return false;
    d.nst = k;
    out->d = d;
    out->E = b > 0 ? 12 : (c > 0 ? 20 : 4);
    out->fast = true;
    return true;
  }
  if (a >= 3 && !(b > 0 && c > 0)) {
    int E;
    // E = 16 (radix-16 stages) only where asked: the y passes run best with it, the
    // z and x passes with E = 8 (fewer registers per lane).  EQ_FFT_E16=0/1 overrides.
    const char* e16 = std::getenv("EQ_FFT_E16");
    const bool use16 = e16 ? (e16[0] == '1') : wide;
    if (b == 0 && c == 0 && a >= 7 && use16) {
      E = 16;
      for (int i = 0; i < a / 4; ++i) d.r[k++] = 16;
      if (a % 4) d.r[k++] = 1 << (a % 4);
    } else {
      E = (b > 0) ? 24 : (c > 0 ? 40 : 8);
      for (int i = 0; i < a / 3; ++i) d.r[k++] = 8;
      if (a % 3) d.r[k++] = 1 << (a % 3);
      for (int i = 0; i < b; ++i) d.r[k++] = 3;
      for (int i = 0; i < c; ++i) d.r[k++] = 5;
    }
    if (k > kMaxStages) return false;
    d.nst = k;
    out->d = d;
    out->E = E;
    out->fast = true;
    return true;
  }
  int q = a / 3, r = a % 3;
  if (r == 1 && q >= 1) { q -= 1; r = 4; }     // 2^(3q+1) = 8^(q-1) * 4 * 4
  for (int i = 0; i < q; ++i) d.r[k++] = 8;
  if (r == 4) { d.r[k++] = 4; d.r[k++] = 4; }
  else if (r == 2) d.r[k++] = 4;
  else if (r == 1) d.r[k++] = 2;
  for (int i = 0; i < b; ++i) d.r[k++] = 3;
  for (int i = 0; i < c; ++i) d.r[k++] = 5;
  if (k > kMaxStages) return false;
  d.nst = k;
  out->d = d;
  out->E = (n % 8 == 0) ? 8 : ((n % 4 == 0) ? 4 : 2);
  out->fast = false;
  return true;
}

eq_status validate(const eq_desc* d) {
  if (!d) return fail(EQ_ERR_ARG, "null descriptor");
  if (d->batch < 1) return fail(EQ_ERR_ARG, "batch must be >= 1");
  if (d->op != EQ_OP_CDO && d->op != EQ_OP_DDO) return fail(EQ_ERR_ARG, "op must be EQ_OP_CDO or EQ_OP_DDO");
  if (d->prec != EQ_FP64 && d->prec != EQ_FP32) return fail(EQ_ERR_ARG, "prec must be EQ_FP64 or EQ_FP32");
  if (!std::isfinite(d->h) || !(d->h > 0.0)) return fail(EQ_ERR_ARG, "h must be finite and > 0");
  if (d->flags & ~(unsigned)(EQ_F_CHECK_FINITE | EQ_F_CAPTURE_GRAPH | EQ_F_OWN_STREAM | EQ_F_PERSISTENT))
    return fail(EQ_ERR_ARG, "unknown or unsupported flag bits");
  AxisFft t;
  const int dims[3] = {d->nx, d->ny, d->nz};
  const char* names[3] = {"nx", "ny", "nz"};
  for (int i = 0; i < 3; ++i)
    if (!factor_axis(dims[i], &t))
      return fail(EQ_ERR_SIZE, std::string(names[i]) + " = " + std::to_string(dims[i]) +
                                   ": grid edges must be even, in [4, 1024], with prime factors in {2, 3, 5}");
  // the fused x pass runs the six component lines of a row in one workgroup
  factor_axis(d->nx, &t);
  if (!t.fast && 6 * (d->nx / t.E) > 1024)
    return fail(EQ_ERR_SIZE, "nx = " + std::to_string(d->nx) +
                                 ": six x-lines need more than 1024 threads (nx / largest of 8, 4, 2 dividing it > 170)");
  // total element count must be addressable by the launch grids
  const double rows = (double)d->batch * (d->nz / 2 + 1) * d->ny;
  if (rows > 2.0e9) return fail(EQ_ERR_SIZE, "batch * (nz/2+1) * ny too large for one launch");
  if ((d->flags & EQ_F_PERSISTENT) &&
      !persist_route_supported(Geom{d->nx, d->ny, d->nz, d->nz / 2 + 1, d->batch}, d->prec == EQ_FP64))
    return fail(EQ_ERR_ARG, "EQ_F_PERSISTENT needs FP32 with nx == ny in {64, 128} and nz in {64, 128, 256}");
  return EQ_OK;
}

size_t elem_size(const eq_desc* d) { return d->prec == EQ_FP64 ? sizeof(double) : sizeof(float); }

// max_q |s(q)|^2 = sum over axes of max_q s_a(q)^2, from the symbol definitions
// (Section 4.1 for CDO, Section 4.2 for DDO).
double symbol_max2(const eq_desc* d) {
  double smax2 = 0.0;
  const int dims[3] = {d->nx, d->ny, d->nz};
  for (int a = 0; a < 3; ++a) {
    double m = 0.0;
    const int n = dims[a];
    for (int q = 0; q < n; ++q) {
      double v;
      if (d->op == EQ_OP_CDO) {
        const int k = (2 * q < n) ? q : ((2 * q == n) ? 0 : q - n);
        v = 2.0 * M_PI * k / (n * d->h);
      } else {
        v = ((2 * q) % n == 0) ? 0.0 : std::sin(2.0 * M_PI * q / n) / d->h;
      }
      m = std::max(m, v * v);
    }
    smax2 += m;
  }
  return smax2;
}


struct Layout {
  size_t w_bytes, sym_bytes, tw64_bytes, tw32_bytes, part_bytes, red_bytes, flag_bytes, ctr_bytes;
  size_t total() const {
    return w_bytes + sym_bytes + tw64_bytes + tw32_bytes + part_bytes + red_bytes + flag_bytes + ctr_bytes;
  }
};

Layout layout_of(const eq_desc* d) {
  Layout L{};
  const size_t nzh = (size_t)d->nz / 2 + 1;
  L.w_bytes = (size_t)d->batch * 6 * nzh * d->ny * d->nx * 2 * elem_size(d);
  const Geom gg{d->nx, d->ny, d->nz, (int)nzh, d->batch};
  if (plane_route_supported(gg, d->prec == EQ_FP64)) {   // three-pass spectrum: x is the half axis
    const size_t w3 = (size_t)d->batch * 6 * d->nz * d->ny * (d->nx / 2 + 1) * 2 * elem_size(d);
    L.w_bytes = std::max(L.w_bytes, w3);
  }
  const size_t ntab = (size_t)d->nx + d->ny + d->nz;
  L.sym_bytes = 2 * ntab * sizeof(double);     // symbols with h, then h-free symbols
  L.tw64_bytes = ntab * sizeof(double2);
  L.tw32_bytes = ntab * sizeof(float2);
  L.part_bytes = (size_t)d->batch * kRedBlocks * kRedWidth * sizeof(double);
  L.red_bytes = 0;   // the per-field records live in pinned host memory (see eq_plan)
  L.flag_bytes = 256;
  // persistent launch: queue head, workgroups done, error flag, spare, then two counters per field
  L.ctr_bytes = (d->flags & EQ_F_PERSISTENT) ? (size_t)(4 + 2 * d->batch) * sizeof(unsigned) : 0;
  return L;
}

enum PassId {
  P_Z_R2C = 0, P_Y_FWD, P_X_PROJ, P_Y_INV, P_Z_C2R, P_DIV_DDO, P_X_DIV, P_Y_INV3, P_Z_C2R3, P_DIV_STATS,
  P_REDUCE, P_CHECK, P_X_FWD, P_PROJ_ONLY, P_PLANE_R2C, P_Z_PROJ, P_PLANE_C2R, P_X_POT, P_PERSIST, P_COUNT
};
const char* kPassNames[P_COUNT] = {
  "z_r2c", "y_fwd", "x_proj", "y_inv", "z_c2r", "div_ddo", "x_div", "y_inv3", "z_c2r3", "div_stats",
  "reduce_final", "check_finite", "x_fwd", "proj_only", "plane_r2c", "z_proj", "plane_c2r", "x_pot", "persist"};

struct TimingRec { int pass; hipEvent_t a, b; };

}  // namespace

struct eq_plan_s {
  eq_desc desc{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Geom g{};
  AxisFft ax{}, ay{}, az{};
  Tune tune{};
  void* W = nullptr;
  double* sym = nullptr;
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
  double* partials = nullptr;
  double* red = nullptr;        // per-field reduction records: pinned host memory ...
  double* red_dev = nullptr;    // ... which the final reduction kernel writes through this alias
  double smax2 = 0.0;           // max_q |s(q)|^2 of the operator's symbol (for the relative residual)
  int* flag = nullptr;
  unsigned* ctr = nullptr;      // persistent launch counters (EQ_F_PERSISTENT)
  // timing
  bool timing = false;
  int timing_pass = -1;      // -1: every pass, else the one pass id bracketed by events
  std::vector<TimingRec> pending;
  std::vector<hipEvent_t> event_pool;
  long long launches[P_COUNT] = {};
  double total_ms[P_COUNT] = {};
  double total_bytes[P_COUNT] = {};
  bool last_removed = false;   // whether the current eq_project writes the removed part
  // graph cache
  struct GraphEntry { const void* in; void* eq; void* rem; hipGraph_t graph; hipGraphExec_t exec; };
  std::vector<GraphEntry> graphs;
};

namespace {

// Symbol tables: sym[0 .. nx+ny+nz) carry 1/h (divergence), the next nx+ny+nz are h-free
// (projection).
const double* sym_unit(const eq_plan_s* p) { return p->sym + (p->g.nx + p->g.ny + p->g.nz); }

// The three-pass z projection with four elements per thread (FP32): asked for, or the persistent
// launch's z stage.
bool zp_e4(const eq_plan_s* p, const Tune& tn) {
  return p->desc.prec == EQ_FP32 && (tn.zp_e == 4 || (p->desc.flags & EQ_F_PERSISTENT));
}

// Whether eq_project takes the three-pass route under tuning tn.
bool use_plane(const eq_plan_s* p, const Tune& tn) {
  if (p->desc.flags & EQ_F_PERSISTENT) return true;          // one persistent launch of the three passes
  if (tn.schedule == 5 || !plane_route_supported(p->g, p->desc.prec == EQ_FP64)) return false;
  // default: three passes where a plane leaves the workgroup room to breathe (nx <= 128);
  // a 256^2 FP32 plane fills a CU's registers and runs no faster than five passes
  return tn.schedule == 3 || p->g.nx <= 128;
}

size_t spectrum_plane_elems(const eq_plan_s* p) { return (size_t)p->g.nzh * p->g.ny * p->g.nx; }
size_t field_elems(const eq_plan_s* p) { return (size_t)p->g.nz * p->g.ny * p->g.nx; }

double pass_bytes(const eq_plan_s* p, int pass) {
  const double es = (double)elem_size(&p->desc);
  const double B = p->g.batch;
  const double M = (double)field_elems(p);
  const double Q = (double)spectrum_plane_elems(p) * 2 * es;   // bytes of one component's half spectrum
  const double Q3 = (double)p->g.nz * p->g.ny * (p->g.nx / 2 + 1) * 2 * es;   // same, half along x
  switch (pass) {
    case P_Z_R2C: return B * 6 * (M * es + Q);
    case P_Y_FWD: case P_X_PROJ: case P_Y_INV: case P_X_FWD: case P_PROJ_ONLY: return B * 6 * 2 * Q;
    case P_Z_C2R: return B * 6 * (Q + M * es) + (p->last_removed ? B * 6 * 2 * M * es : 0.0);
    case P_PLANE_R2C: return B * 6 * (M * es + Q3);
    case P_Z_PROJ: return B * 6 * 2 * Q3;
    case P_PLANE_C2R: return B * 6 * (Q3 + M * es) + (p->last_removed ? B * 6 * 2 * M * es : 0.0);
    case P_PERSIST:     // the three passes
      return B * 6 * (M * es + Q3) + B * 6 * 2 * Q3 + B * 6 * (Q3 + M * es) +
             (p->last_removed ? B * 6 * 2 * M * es : 0.0);
    case P_DIV_DDO: return B * 6 * M * es;
    case P_X_DIV: case P_X_POT: return B * (6 * Q + 3 * Q);
    case P_Y_INV3: return B * 3 * 2 * Q;
    case P_Z_C2R3: return B * 3 * (Q + M * es);
    case P_DIV_STATS: return B * 9 * M * es;
    case P_CHECK: return B * 6 * M * es;
    default: return 0.0;
  }
}

hipEvent_t get_event(eq_plan_s* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket one launch with events when timing is on.
template <typename F>
hipError_t timed(eq_plan_s* p, int pass, F&& launch, double frac = 1.0) {
  if (!p->timing || (p->timing_pass >= 0 && pass != p->timing_pass)) return launch();
  hipEvent_t a = get_event(p), b = get_event(p);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, p->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, p->stream);
  if (e != hipSuccess) return e;
  p->pending.push_back({pass, a, b});
  p->total_bytes[pass] += frac * pass_bytes(p, pass);
  if (p->pending.size() > 4096) {     // bound the backlog: fold completed records
    (void)hipEventSynchronize(b);
    for (auto& r : p->pending) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, r.a, r.b);
      p->total_ms[r.pass] += ms;
      p->launches[r.pass] += 1;
      p->event_pool.push_back(r.a);
      p->event_pool.push_back(r.b);
    }
    p->pending.clear();
  }
  return hipSuccess;
}

void drop_graphs(eq_plan_s* p) {
  for (auto& ge : p->graphs) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    if (ge.graph) (void)hipGraphDestroy(ge.graph);
  }
  p->graphs.clear();
}

void release(eq_plan_s* p) {
  if (!p) return;
  drop_graphs(p);
  for (auto& r : p->pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : p->event_pool) (void)hipEventDestroy(e);
  if (p->W) (void)hipFree(p->W);
  if (p->sym) (void)hipFree(p->sym);
  if (p->tw64) (void)hipFree(p->tw64);
  if (p->tw32) (void)hipFree(p->tw32);
  if (p->partials) (void)hipFree(p->partials);
  if (p->red) (void)hipHostFree(p->red);
  if (p->flag) (void)hipFree(p->flag);
  if (p->ctr) (void)hipFree(p->ctr);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

eq_status dev_alloc(void** ptr, size_t bytes, const char* what) {
  if (fault_inject_alloc()) return fail(EQ_ERR_NOMEM, std::string("injected allocation failure: ") + what);
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(EQ_ERR_NOMEM, std::string("hipMalloc(") + what + ", " + std::to_string(bytes) + " B): " +
                                  hipGetErrorString(e));
  }
  return EQ_OK;
}

// Launch shapes of a tuning against the grid and the device limits.
eq_status check_shapes(const eq_plan_s* p, const Tune& tn) {
  int limit = 0;
  EQ_HIP(hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device), "hipDeviceGetAttribute");
  const Geom& g = p->g;
  const int eb = 2 * (int)elem_size(&p->desc);
  const int ty = pick_tx_y(g, p->ay, eb, tn), tz = pick_tx_z(g, p->az, eb, tn), rw = pick_rw_x(g, p->ax, eb, tn);
  auto round64 = [](int t) { return ((t + 63) / 64) * 64; };
  const int thy = ty * (g.ny / p->ay.E), thz = (tz / 2) * (g.nz / p->az.E);
  const int thx = x_threads_per_row(p->ax, eb, tn) * rw;
  if (ty < 1 || g.nx % ty || round64(thy) > max_threads(p->ay)) return fail(EQ_ERR_ARG, "tx_y does not fit this grid");
  if (tz < 2 || (tz & 1) || g.nx % tz || round64(thz) > max_threads(p->az))
    return fail(EQ_ERR_ARG, "tx_z does not fit this grid");
  if (rw < 1 || round64(thx) > max_threads(p->ax)) return fail(EQ_ERR_ARG, "rw_x does not fit this grid");
  // the radix-4 schedules of 3/5-smooth edges (E = 12, 20) exist for the split x kernel only
  if (p->ax.fast && (p->ax.E == 12 || p->ax.E == 20) && !x_split(p->ax, eb, tn))
    return fail(EQ_ERR_ARG, "radix4 on a 3/5-smooth x edge needs the split x kernel (xsplit 0 or 2)");
  if (tn.chunk < -1 || tn.chunk > g.batch * g.nzh) return fail(EQ_ERR_ARG, "chunk out of range");
  if (tn.schedule != 0 && tn.schedule != 3 && tn.schedule != 5) return fail(EQ_ERR_ARG, "schedule must be 0, 3 or 5");
  const bool fp64 = p->desc.prec == EQ_FP64;
  if (tn.schedule == 3 && !plane_route_supported(g, fp64))
    return fail(EQ_ERR_ARG, "the three-pass schedule needs nx == ny in {64, 128, 256} (FP64: 64, 128) and nz in "
                            "{64, 128, 256}");
  size_t need = std::max(lds_y(g, p->ay, eb, tn), std::max(lds_z(g, p->az, eb, tn), lds_x(g, p->ax, eb, tn)));
  if (use_plane(p, tn)) {
    const int tc = pick_tc_zproj(g, fp64, tn.tc_zp, zp_e4(p, tn));
    if (tn.tc_zp < 0 || (tn.tc_zp > 0 && tc != tn.tc_zp)) return fail(EQ_ERR_ARG, "tc_zp does not fit this grid");
    need = std::max(need, std::max(plane_lds(g, fp64), zproj_lds(g, fp64, tc)));
  }
  if (need > (size_t)limit)
    return fail(EQ_ERR_SIZE, "grid needs " + std::to_string(need) + " B of LDS per workgroup; device allows " +
                                 std::to_string(limit));
  return EQ_OK;
}

// Tuning from the environment: EQ_TUNE="tx_y=16,tx_z=32,rw_x=4,chunk=32" (any subset).
Tune tune_from_env() {
  Tune t;
  const char* v = std::getenv("EQ_TUNE");
  if (!v) return t;
  std::string s(v);
  size_t pos = 0;
  while (pos < s.size()) {
    size_t end = s.find_first_of(", ", pos);
    if (end == std::string::npos) end = s.size();
    const std::string kv = s.substr(pos, end - pos);
    const size_t eqp = kv.find('=');
    if (eqp != std::string::npos) {
      const std::string key = kv.substr(0, eqp);
      const int val = std::atoi(kv.c_str() + eqp + 1);
      if (key == "tx_y") t.tx_y = val;
      else if (key == "tx_z") t.tx_z = val;
      else if (key == "rw_x") t.rw_x = val;
      else if (key == "chunk") t.chunk = val;
      else if (key == "radix16") t.radix16 = val;
      else if (key == "radix4") t.radix4 = val;
      else if (key == "xsplit") t.xsplit = val;
      else if (key == "schedule") t.schedule = val;
      else if (key == "tc_zp") t.tc_zp = val;
      else if (key == "zp_e") t.zp_e = val;
    }
    pos = end + 1;
  }
  return t;
}

// Radix schedules of the three axes for a radix-16 mask (-1: y only); radix4 = 1 puts the x
// axis on radix-4 stages where the six-component x kernel serves it (FP32, powers of two
// 32 .. 512), and is ignored elsewhere.
void set_axes(eq_plan_s* p, int mask, int radix4 = 0, int xsplit = 0) {
  if (mask < 0) mask = 2;
  const int nx = p->desc.nx;
  // radix 4 on a 3/5-smooth x axis has only the split kernel's schedules (E = 12 or 20)
  const bool pow2 = (nx & (nx - 1)) == 0;
  const bool x4 = radix4 == 1 && (pow2 || xsplit != 1) && x6_radix4_available(nx, p->desc.prec == EQ_FP64);
  factor_axis(nx, &p->ax, (mask & 1) != 0, x4);
  // the one-line-per-thread-group x pass needs 6 * nx / E threads in one workgroup: past 512
  // (nx = 1024 on radix 8) take radix 16
  if (p->ax.fast && p->ax.E == 8 && 6 * (nx / 8) > 512) factor_axis(nx, &p->ax, true);
  factor_axis(p->desc.ny, &p->ay, (mask & 2) != 0);
  factor_axis(p->desc.nz, &p->az, (mask & 4) != 0);
}

// Planes per chunk of the y/x/y sequence (the whole range when chunking is off).
int chunk_planes(const eq_plan_s* p) {
  const int total = p->g.batch * p->g.nzh;
  if (p->tune.chunk > 0) return std::min(p->tune.chunk, total);
  return total;
}

template <typename T>
eq_status run_project_plane(eq_plan_s* p, const void* s_in, void* s_eq, void* s_removed) {
  using C = cplx<T>;
  C* W = static_cast<C*>(p->W);
  const C* tw = reinterpret_cast<const C*>(sizeof(T) == 8 ? (const void*)p->tw64 : (const void*)p->tw32);
  const C* twx = tw;
  const C* twy = tw + p->g.nx;
  const C* twz = tw + p->g.nx + p->g.ny;
  const Geom& g = p->g;
  hipStream_t s = p->stream;
  const int tc = pick_tc_zproj(g, p->desc.prec == EQ_FP64, p->tune.tc_zp, zp_e4(p, p->tune));
  EQ_HIP(timed(p, P_PLANE_R2C, [&] { return launch_plane_r2c<T>(static_cast<const T*>(s_in), W, g, twx, twy, s); }),
         "plane_r2c launch");
  EQ_HIP(timed(p, P_Z_PROJ, [&] { return launch_zproj<T>(W, g, twz, sym_unit(p), tc, zp_e4(p, p->tune), s); }),
         "z_proj launch");
  EQ_HIP(timed(p, P_PLANE_C2R, [&] {
           return launch_plane_c2r<T>(W, static_cast<T*>(s_eq), static_cast<const T*>(s_in), static_cast<T*>(s_removed),
                                      g, twx, twy, s);
         }),
         "plane_c2r launch");
  return EQ_OK;
}

// EQ_F_PERSISTENT: the three passes as one launch over a device-side work queue.
template <typename T>
eq_status run_project_persist(eq_plan_s* p, const void* s_in, void* s_eq, void* s_removed) {
  using C = cplx<T>;
  C* W = static_cast<C*>(p->W);
  const C* tw = reinterpret_cast<const C*>(sizeof(T) == 8 ? (const void*)p->tw64 : (const void*)p->tw32);
  const Geom& g = p->g;
  EQ_HIP(timed(p, P_PERSIST, [&] {
           return launch_persist<T>(static_cast<const T*>(s_in), W, static_cast<T*>(s_eq), static_cast<T*>(s_removed), g,
                                    tw, tw + g.nx, tw + g.nx + g.ny, sym_unit(p), p->ctr, p->stream);
         }),
         "persistent launch");
  return EQ_OK;
}

// e.on: the real fields are a sample embedded in the box (five passes; the z passes read
// the sample with a zero buffer around it and write the sample's voxels only).
template <typename T>
eq_status run_project(eq_plan_s* p, const void* s_in, void* s_eq, void* s_removed, const Embed& e = Embed{}) {
  using C = cplx<T>;
  if constexpr (sizeof(T) == 4) {
    if (!e.on && (p->desc.flags & EQ_F_PERSISTENT)) return run_project_persist<T>(p, s_in, s_eq, s_removed);
  }
  if (!e.on && use_plane(p, p->tune)) return run_project_plane<T>(p, s_in, s_eq, s_removed);
  C* W = static_cast<C*>(p->W);
  const C* tw = reinterpret_cast<const C*>(sizeof(T) == 8 ? (const void*)p->tw64 : (const void*)p->tw32);
  const C* twx = tw;
  const C* twy = tw + p->g.nx;
  const C* twz = tw + p->g.nx + p->g.ny;
  const Geom& g = p->g;
  hipStream_t s = p->stream;
  const size_t M = field_elems(p);
  EQ_HIP(timed(p, P_Z_R2C,
               [&] { return launch_z_r2c<T>(static_cast<const T*>(s_in), W, g, p->az, twz, p->tune, s, e); }),
         "z_r2c launch");
  const int total = g.batch * g.nzh, cp = chunk_planes(p);
  for (int pl0 = 0; pl0 < total; pl0 += cp) {
    const int npl = std::min(cp, total - pl0);
    const double frac = (double)npl / (double)total;    // share of the field's bytes in this launch
    EQ_HIP(timed(p, P_Y_FWD, [&] { return launch_y<T>(W, g, pl0, npl, 6, p->ay, twy, false, p->tune, s); }, frac),
           "y_fwd launch");
    EQ_HIP(timed(
               p, P_X_PROJ,
               [&] { return launch_x<T>(W, g, pl0, npl, XM_FWD | XM_PROJ | XM_INV, p->ax, twx, sym_unit(p), p->tune, s); },
               frac),
           "x_proj launch");
    EQ_HIP(timed(p, P_Y_INV, [&] { return launch_y<T>(W, g, pl0, npl, 6, p->ay, twy, true, p->tune, s); }, frac),
           "y_inv launch");
  }
  const size_t Mo = e.on ? (size_t)g.nz * e.ny0 * e.nx0 : M;      // voxels of one output component
  EQ_HIP(timed(p, P_Z_C2R, [&] {
           return launch_z_c2r<T>(W, static_cast<T*>(s_eq), 6 * Mo, Mo, static_cast<const T*>(s_in),
                                  static_cast<T*>(s_removed), 6, g, p->az, twz, p->tune, s, e);
         }),
         "z_c2r launch");
  return EQ_OK;
}

// Potential of the removed part: forward transform of the six components, the per-frequency
// potential (three components) in the x pass, inverse transform of those three into y_out.
template <typename T>
eq_status run_potential(eq_plan_s* p, const void* s_in, void* y_out) {
  using C = cplx<T>;
  const Geom& g = p->g;
  hipStream_t st = p->stream;
  const size_t M = field_elems(p);
  C* W = static_cast<C*>(p->W);
  const C* tw = reinterpret_cast<const C*>(sizeof(T) == 8 ? (const void*)p->tw64 : (const void*)p->tw32);
  const C* twx = tw;
  const C* twy = tw + g.nx;
  const C* twz = tw + g.nx + g.ny;
  const int total = g.batch * g.nzh;
  EQ_HIP(timed(p, P_Z_R2C, [&] { return launch_z_r2c<T>(static_cast<const T*>(s_in), W, g, p->az, twz, p->tune, st); }),
         "z_r2c launch");
  EQ_HIP(timed(p, P_Y_FWD, [&] { return launch_y<T>(W, g, 0, total, 6, p->ay, twy, false, p->tune, st); }),
         "y_fwd launch");
  EQ_HIP(timed(p, P_X_POT, [&] {
           return launch_x<T>(W, g, 0, total, XM_FWD | XM_DISP | XM_INV, p->ax, twx, sym_unit(p), p->tune, st,
                              p->desc.h);
         }),
         "x_pot launch");
  EQ_HIP(timed(p, P_Y_INV3, [&] { return launch_y<T>(W, g, 0, total, 3, p->ay, twy, true, p->tune, st); }),
         "y_inv3 launch");
  EQ_HIP(timed(p, P_Z_C2R3, [&] {
           return launch_z_c2r<T>(W, static_cast<T*>(y_out), 3 * M, M, nullptr, nullptr, 3, g, p->az, twz, p->tune, st);
         }),
         "z_c2r3 launch");
  return EQ_OK;
}

template <typename T>
eq_status run_check_finite(eq_plan_s* p, const void* s_in, size_t n_override = 0) {
  const size_t n = n_override ? n_override : (size_t)p->g.batch * 6 * field_elems(p);
  EQ_HIP(launch_fill_int(p->flag, 1, 0, p->stream), "fill launch");
  EQ_HIP(timed(p, P_CHECK, [&] { return launch_check_finite<T>(static_cast<const T*>(s_in), n, p->flag, p->stream); }),
         "check_finite launch");
  int h = 0;
  EQ_HIP(hipMemcpyAsync(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream), "hipMemcpyAsync");
  EQ_HIP(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  if (h) return fail(EQ_ERR_NONFINITE, "input holds a NaN or Inf");
  return EQ_OK;
}

template <typename T>
eq_status run_residual(eq_plan_s* p, const void* s, double* norms, void* div_out) {
  using C = cplx<T>;
  const Geom& g = p->g;
  hipStream_t st = p->stream;
  const size_t M = field_elems(p);
  if (p->desc.op == EQ_OP_DDO) {
    EQ_HIP(timed(p, P_DIV_DDO, [&] {
             return launch_div_ddo<T>(static_cast<const T*>(s), static_cast<T*>(div_out), p->partials, kRedBlocks, g,
                                      p->desc.h, st);
           }),
           "div_ddo launch");
  } else {
    C* W = static_cast<C*>(p->W);
    const C* tw = reinterpret_cast<const C*>(sizeof(T) == 8 ? (const void*)p->tw64 : (const void*)p->tw32);
    const C* twx = tw;
    const C* twy = tw + g.nx;
    const C* twz = tw + g.nx + g.ny;
    const size_t Q = spectrum_plane_elems(p);
    // divergence field destination: the caller's buffer, else the upper half of each field's workspace
    T* dst = static_cast<T*>(div_out);
    size_t dfield = 3 * M, dcomp = M;
    if (!dst) {
      dst = reinterpret_cast<T*>(W + 3 * Q);
      dfield = 2 * 6 * Q;
    }
    EQ_HIP(timed(p, P_Z_R2C, [&] { return launch_z_r2c<T>(static_cast<const T*>(s), W, g, p->az, twz, p->tune, st); }),
           "z_r2c launch");
    const int total = g.batch * g.nzh;
    EQ_HIP(timed(p, P_Y_FWD, [&] { return launch_y<T>(W, g, 0, total, 6, p->ay, twy, false, p->tune, st); }),
           "y_fwd launch");
    EQ_HIP(timed(p, P_X_DIV, [&] {
             return launch_x<T>(W, g, 0, total, XM_FWD | XM_DIV | XM_INV, p->ax, twx, p->sym, p->tune, st);
           }),
           "x_div launch");
    EQ_HIP(timed(p, P_Y_INV3, [&] { return launch_y<T>(W, g, 0, total, 3, p->ay, twy, true, p->tune, st); }),
           "y_inv3 launch");
    EQ_HIP(timed(p, P_Z_C2R3, [&] {
             return launch_z_c2r<T>(W, dst, dfield, dcomp, nullptr, nullptr, 3, g, p->az, twz, p->tune, st);
           }),
           "z_c2r3 launch");
    EQ_HIP(timed(p, P_DIV_STATS, [&] {
             return launch_div_stats<T>(dst, dfield, dcomp, static_cast<const T*>(s), p->partials, kRedBlocks, g, st);
           }),
           "div_stats launch");
  }
  const int nred = p->desc.op == EQ_OP_DDO ? div_ddo_blocks(g, kRedBlocks, p->desc.prec == EQ_FP64) : kRedBlocks;
  EQ_HIP(timed(p, P_REDUCE, [&] { return launch_reduce_final(p->partials, nred, g.batch, p->red_dev, st); }),
         "reduce launch");
  EQ_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (p->ctr) {
    // a persistent launch whose dependency wait gave up (never expected) is reported here
    unsigned gave_up = 0;
    EQ_HIP(hipMemcpy(&gave_up, p->ctr + 2, sizeof(unsigned), hipMemcpyDeviceToHost), "hipMemcpy(counters)");
    if (gave_up) return fail(EQ_ERR_DEVICE, "a persistent projection's dependency wait gave up; its output is invalid and the plan must be destroyed");
  }
  const double* host = p->red;
  const double smax2 = p->smax2;
  const double w[6] = {1, 1, 1, 2, 2, 2};
  for (int b = 0; b < g.batch; ++b) {
    const double* r = &host[(size_t)b * kRedWidth];
    // ||S - c0||_F^2 from sums of d = S - shift (shift: the field's first voxel), so a mean
    // far above the spread does not cancel
    double dev2 = 0.0;
    for (int c = 0; c < 6; ++c) dev2 += w[c] * (r[8 + c] - r[2 + c] * r[2 + c] / (double)M);
    const double l2 = std::sqrt(r[0]);
    const double denom = std::sqrt(smax2) * std::sqrt(std::max(dev2, 0.0));
    norms[3 * b + 0] = l2;
    norms[3 * b + 1] = std::sqrt(r[1]);
    norms[3 * b + 2] = denom > 0.0 ? l2 / denom : 0.0;
  }
  return EQ_OK;
}

// [a, a + abytes) and [b, b + bbytes) share a byte
bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + bbytes && y < x + abytes;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() { if (prev >= 0) (void)hipSetDevice(prev); }
};

}  // namespace

// =================================================================== ABI ====

extern "C" {

const char* eq_status_str(eq_status s) {
  // C callers may pass any int; read it as one (a C++ load of an out-of-range enum value is undefined)
  int v = 0;
  std::memcpy(&v, &s, sizeof(v) < sizeof(s) ? sizeof(v) : sizeof(s));
  switch (v) {
    case EQ_OK: return "EQ_OK";
    case EQ_ERR_ARG: return "EQ_ERR_ARG";
    case EQ_ERR_SIZE: return "EQ_ERR_SIZE";
    case EQ_ERR_NOMEM: return "EQ_ERR_NOMEM";
    case EQ_ERR_DEVICE: return "EQ_ERR_DEVICE";
    case EQ_ERR_NONFINITE: return "EQ_ERR_NONFINITE";
  }
  return "EQ_ERR_UNKNOWN";
}

const char* eq_last_error(void) { return g_last_error.c_str(); }

const char* eq_version(void) { return "libeq 0.1 gfx950"; }

eq_status eq_plan_footprint(const eq_desc* d, size_t* bytes) {
  if (!bytes) return fail(EQ_ERR_ARG, "null output pointer");
  eq_status st = validate(d);
  if (st != EQ_OK) return st;
  *bytes = layout_of(d).total();
  return EQ_OK;
}

eq_status eq_plan(const eq_desc* d, void* hip_stream, eq_plan_t* out) {
  if (!out) return fail(EQ_ERR_ARG, "null plan output pointer");
  *out = nullptr;
  eq_status st = validate(d);
  if (st != EQ_OK) return st;
  eq_plan_s* p = new (std::nothrow) eq_plan_s();
  if (!p) return fail(EQ_ERR_NOMEM, "host allocation failed");
  p->desc = *d;
  p->g = Geom{d->nx, d->ny, d->nz, d->nz / 2 + 1, d->batch};
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { release(p); return hip_fail(e, "hipGetDevice"); }
  p->tune = tune_from_env();
  set_axes(p, p->tune.radix16, p->tune.radix4, p->tune.xsplit);
  if ((st = check_shapes(p, p->tune)) != EQ_OK) { release(p); return st; }
  if (d->flags & EQ_F_OWN_STREAM) {
    e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e != hipSuccess) { release(p); return hip_fail(e, "hipStreamCreateWithFlags"); }
    p->own_stream = true;
  } else {
    p->stream = static_cast<hipStream_t>(hip_stream);
  }
  const Layout L = layout_of(d);
  if ((st = dev_alloc(&p->W, L.w_bytes, "workspace")) != EQ_OK ||
      (st = dev_alloc((void**)&p->sym, L.sym_bytes, "symbols")) != EQ_OK ||
      (st = dev_alloc((void**)&p->tw64, L.tw64_bytes, "twiddles64")) != EQ_OK ||
      (st = dev_alloc((void**)&p->tw32, L.tw32_bytes, "twiddles32")) != EQ_OK ||
      (st = dev_alloc((void**)&p->partials, L.part_bytes, "partials")) != EQ_OK ||
      (st = dev_alloc((void**)&p->flag, L.flag_bytes, "flag")) != EQ_OK ||
      (L.ctr_bytes && (st = dev_alloc((void**)&p->ctr, L.ctr_bytes, "persistent counters")) != EQ_OK)) {
    release(p);
    return st;
  }
  if (p->ctr) {
    e = launch_fill_int(reinterpret_cast<int*>(p->ctr), (int)(L.ctr_bytes / sizeof(unsigned)), 0, p->stream);
    if (e != hipSuccess) { release(p); return hip_fail(e, "counter fill launch"); }
  }
  // the residual's per-field records go straight to pinned, device-mapped host memory:
  // no copy engine and no pageable staging between the last kernel and the host
  e = hipHostMalloc((void**)&p->red, (size_t)d->batch * kRedWidth * sizeof(double),
                    hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) { p->red = nullptr; release(p); return hip_fail(e, "hipHostMalloc(reduction records)"); }
  e = hipHostGetDevicePointer((void**)&p->red_dev, p->red, 0);
  if (e != hipSuccess) { release(p); return hip_fail(e, "hipHostGetDevicePointer(reduction records)"); }
  p->smax2 = symbol_max2(d);
  e = launch_tables(p->g, d->op, d->h, p->sym, p->tw64, p->tw32, p->stream);
  if (e != hipSuccess) { release(p); return hip_fail(e, "table kernel launch"); }
  *out = p;
  return EQ_OK;
}

eq_status eq_plan_destroy(eq_plan_t p) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  DeviceGuard dg(p->device);
  (void)hipStreamSynchronize(p->stream);
  release(p);
  return EQ_OK;
}

eq_status eq_plan_set_stream(eq_plan_t p, void* hip_stream) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  DeviceGuard dg(p->device);
  drop_graphs(p);
  if (p->own_stream) {
    (void)hipStreamSynchronize(p->stream);
    (void)hipStreamDestroy(p->stream);
    p->own_stream = false;
  }
  p->stream = static_cast<hipStream_t>(hip_stream);
  return EQ_OK;
}

eq_status eq_project(eq_plan_t p, const void* s_in, void* s_eq, void* s_removed) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  if (!s_in || !s_eq) return fail(EQ_ERR_ARG, "null input or output pointer");
  const size_t bytes = (size_t)p->g.batch * 6 * field_elems(p) * elem_size(&p->desc);
  if (s_removed && (ranges_overlap(s_removed, bytes, s_in, bytes) || ranges_overlap(s_removed, bytes, s_eq, bytes)))
    return fail(EQ_ERR_ARG, "s_removed overlaps s_in or s_eq");
  if (s_eq != s_in && ranges_overlap(s_eq, bytes, s_in, bytes))
    return fail(EQ_ERR_ARG, "s_eq partially overlaps s_in");
  DeviceGuard dg(p->device);
  const bool fp64 = p->desc.prec == EQ_FP64;
  p->last_removed = s_removed != nullptr;
  if (p->desc.flags & EQ_F_CHECK_FINITE) {
    eq_status st = fp64 ? run_check_finite<double>(p, s_in) : run_check_finite<float>(p, s_in);
    if (st != EQ_OK) return st;
  }
  if ((p->desc.flags & EQ_F_CAPTURE_GRAPH) && p->stream == nullptr)
    return fail(EQ_ERR_ARG, "EQ_F_CAPTURE_GRAPH needs a stream other than the null stream");
  const bool use_graph = (p->desc.flags & EQ_F_CAPTURE_GRAPH) && !p->timing;
  if (!use_graph) return fp64 ? run_project<double>(p, s_in, s_eq, s_removed) : run_project<float>(p, s_in, s_eq, s_removed);
  for (auto& ge : p->graphs)
    if (ge.in == s_in && ge.eq == s_eq && ge.rem == s_removed) {
      EQ_HIP(hipGraphLaunch(ge.exec, p->stream), "hipGraphLaunch");
      return EQ_OK;
    }
  eq_plan_s::GraphEntry ge{s_in, s_eq, s_removed, nullptr, nullptr};
  EQ_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  eq_status st = fp64 ? run_project<double>(p, s_in, s_eq, s_removed) : run_project<float>(p, s_in, s_eq, s_removed);
  hipError_t e = hipStreamEndCapture(p->stream, &ge.graph);
  if (st != EQ_OK) { if (ge.graph) (void)hipGraphDestroy(ge.graph); return st; }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) { (void)hipGraphDestroy(ge.graph); return hip_fail(e, "hipGraphInstantiate"); }
  if (p->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(p->graphs.front().exec);
    (void)hipGraphDestroy(p->graphs.front().graph);
    p->graphs.erase(p->graphs.begin());
  }
  p->graphs.push_back(ge);
  EQ_HIP(hipGraphLaunch(ge.exec, p->stream), "hipGraphLaunch");
  return EQ_OK;
}

eq_status eq_project_embedded(eq_plan_t p, const eq_embed* em, const void* s_in, void* s_eq, void* s_removed) {
  if (!p || !em) return fail(EQ_ERR_ARG, "null plan or embedding");
  if (!s_in || !s_eq) return fail(EQ_ERR_ARG, "null input or output pointer");
  const Geom& g = p->g;
  if (em->nx0 < 1 || em->ny0 < 1 || em->ox < 0 || em->oy < 0 || em->ox + em->nx0 > g.nx || em->oy + em->ny0 > g.ny)
    return fail(EQ_ERR_ARG, "the sample (nx0, ny0) at (ox, oy) must lie inside the plan's (nx, ny)");
  Embed e;
  e.nx0 = em->nx0; e.ny0 = em->ny0; e.ox = em->ox; e.oy = em->oy; e.on = true;
  const size_t n = (size_t)g.batch * 6 * g.nz * e.ny0 * e.nx0;
  const size_t bytes = n * elem_size(&p->desc);
  if (s_removed && (ranges_overlap(s_removed, bytes, s_in, bytes) || ranges_overlap(s_removed, bytes, s_eq, bytes)))
    return fail(EQ_ERR_ARG, "s_removed overlaps s_in or s_eq");
  if (s_eq != s_in && ranges_overlap(s_eq, bytes, s_in, bytes)) return fail(EQ_ERR_ARG, "s_eq partially overlaps s_in");
  DeviceGuard dg(p->device);
  const bool fp64 = p->desc.prec == EQ_FP64;
  p->last_removed = s_removed != nullptr;
  if (p->desc.flags & EQ_F_CHECK_FINITE) {
    eq_status st = fp64 ? run_check_finite<double>(p, s_in, n) : run_check_finite<float>(p, s_in, n);
    if (st != EQ_OK) return st;
  }
  return fp64 ? run_project<double>(p, s_in, s_eq, s_removed, e) : run_project<float>(p, s_in, s_eq, s_removed, e);
}

eq_status eq_residual(eq_plan_t p, const void* s, double* norms_host, void* div_out) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  if (!s || !norms_host) return fail(EQ_ERR_ARG, "null field or norms pointer");
  const size_t es = elem_size(&p->desc);
  const size_t fbytes = (size_t)p->g.batch * field_elems(p) * es;     // one component of every field
  if (div_out && ranges_overlap(div_out, 3 * fbytes, s, 6 * fbytes)) return fail(EQ_ERR_ARG, "div_out overlaps the field");
  DeviceGuard dg(p->device);
  return p->desc.prec == EQ_FP64 ? run_residual<double>(p, s, norms_host, div_out)
                                 : run_residual<float>(p, s, norms_host, div_out);
}

eq_status eq_residual_noalloc(const eq_desc* d, void* hip_stream, const void* s, double* norms_dev, void* div_out) {
  eq_status st = validate(d);
  if (st != EQ_OK) return st;
  if (d->op != EQ_OP_DDO)
    return fail(EQ_ERR_ARG, "eq_residual_noalloc: DDO operator only (the CDO residual needs a plan's spectrum workspace)");
  if (!s || !norms_dev) return fail(EQ_ERR_ARG, "null field or norms pointer");
  if (d->batch > kNoAllocFields)
    return fail(EQ_ERR_SIZE, "eq_residual_noalloc: batch " + std::to_string(d->batch) + " exceeds the maximum of " +
                                 std::to_string(kNoAllocFields) + " fields of its static scratch");
  const size_t es = elem_size(d);
  const size_t M = (size_t)d->nx * d->ny * d->nz;
  const size_t bytes = (size_t)d->batch * 6 * M * es;
  const uintptr_t xs = (uintptr_t)s;
  auto hits_field = [&](const void* q, size_t qbytes) {
    const uintptr_t xq = (uintptr_t)q;
    return xq < xs + bytes && xs < xq + qbytes;
  };
  if (div_out && hits_field(div_out, (size_t)d->batch * 3 * M * es)) return fail(EQ_ERR_ARG, "div_out overlaps the field");
  if (hits_field(norms_dev, (size_t)d->batch * 3 * sizeof(double))) return fail(EQ_ERR_ARG, "norms_dev overlaps the field");
  const Geom g{d->nx, d->ny, d->nz, d->nz / 2 + 1, d->batch};
  double* scr = nullptr;
  EQ_HIP(noalloc_scratch(&scr), "hipGetSymbolAddress(scratch)");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const bool fp64 = d->prec == EQ_FP64;
  if (fp64) {
    EQ_HIP(launch_div_ddo<double>(static_cast<const double*>(s), static_cast<double*>(div_out), scr, kRedBlocks, g,
                                  d->h, stream),
           "div_ddo launch");
  } else {
    EQ_HIP(launch_div_ddo<float>(static_cast<const float*>(s), static_cast<float*>(div_out), scr, kRedBlocks, g, d->h,
                                 stream),
           "div_ddo launch");
  }
  const int nred = div_ddo_blocks(g, kRedBlocks, fp64);
  EQ_HIP(launch_reduce_norms(scr, nred, d->batch, 1.0 / (double)M, std::sqrt(symbol_max2(d)), norms_dev, stream),
         "reduce launch");
  return EQ_OK;
}

eq_status eq_potential(eq_plan_t p, const void* s_in, void* y_out) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  if (!s_in || !y_out) return fail(EQ_ERR_ARG, "null field or output pointer");
  const size_t es = elem_size(&p->desc);
  const size_t M = field_elems(p);
  const size_t in_bytes = (size_t)p->g.batch * 6 * M * es, out_bytes = (size_t)p->g.batch * 3 * M * es;
  const uintptr_t x = (uintptr_t)s_in, y = (uintptr_t)y_out;
  if (y < x + in_bytes && x < y + out_bytes) return fail(EQ_ERR_ARG, "y_out overlaps the field");
  DeviceGuard dg(p->device);
  if (p->desc.flags & EQ_F_CHECK_FINITE) {
    const eq_status st = p->desc.prec == EQ_FP64 ? run_check_finite<double>(p, s_in) : run_check_finite<float>(p, s_in);
    if (st != EQ_OK) return st;
  }
  return p->desc.prec == EQ_FP64 ? run_potential<double>(p, s_in, y_out) : run_potential<float>(p, s_in, y_out);
}

eq_status eq_plan_tune(eq_plan_t p, const eq_tune* tv) {
  if (!p || !tv) return fail(EQ_ERR_ARG, "null pointer");
  if (tv->tx_y < 0 || tv->tx_z < 0 || tv->rw_x < 0) return fail(EQ_ERR_ARG, "negative launch shape");
  if (tv->radix16 < -1 || tv->radix16 > 7) return fail(EQ_ERR_ARG, "radix16 must be -1 or a mask of 1|2|4");
  if (tv->radix4 != 0 && tv->radix4 != 1) return fail(EQ_ERR_ARG, "radix4 must be 0 or 1 (x axis)");
  if (tv->xsplit < 0 || tv->xsplit > 2) return fail(EQ_ERR_ARG, "xsplit must be 0, 1 or 2");
  if (tv->zp_e != 0 && tv->zp_e != 4 && tv->zp_e != 8) return fail(EQ_ERR_ARG, "zp_e must be 0, 4 or 8");
  Tune t;
  t.tx_y = tv->tx_y; t.tx_z = tv->tx_z; t.rw_x = tv->rw_x; t.chunk = tv->chunk;
  t.radix16 = tv->radix16;
  t.radix4 = tv->radix4;
  t.xsplit = tv->xsplit;
  t.schedule = tv->schedule;
  t.tc_zp = tv->tc_zp;
  t.zp_e = tv->zp_e;
  DeviceGuard dg(p->device);
  const AxisFft ax = p->ax, ay = p->ay, az = p->az;
  set_axes(p, t.radix16, t.radix4, t.xsplit);
  eq_status st = check_shapes(p, t);
  if (st != EQ_OK) {
    p->ax = ax; p->ay = ay; p->az = az;
    return st;
  }
  EQ_HIP(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  drop_graphs(p);
  p->tune = t;
  return EQ_OK;
}

eq_status eq_plan_get_tune(eq_plan_t p, eq_tune* t) {
  if (!p || !t) return fail(EQ_ERR_ARG, "null pointer");
  const int eb = 2 * (int)elem_size(&p->desc);
  t->tx_y = pick_tx_y(p->g, p->ay, eb, p->tune);
  t->tx_z = pick_tx_z(p->g, p->az, eb, p->tune);
  t->rw_x = pick_rw_x(p->g, p->ax, eb, p->tune);
  t->chunk = chunk_planes(p);
  t->radix16 = (p->ax.E == 16 ? 1 : 0) | (p->ay.E == 16 ? 2 : 0) | (p->az.E == 16 ? 4 : 0);
  t->radix4 = (p->ax.E == 4 || p->ax.E == 12 || p->ax.E == 20) ? 1 : 0;
  t->xsplit = x_split(p->ax, eb, p->tune) ? 2 : 1;
  const bool plane = use_plane(p, p->tune);
  t->schedule = plane ? 3 : 5;
  t->tc_zp = plane ? pick_tc_zproj(p->g, p->desc.prec == EQ_FP64, p->tune.tc_zp, zp_e4(p, p->tune)) : 0;
  t->zp_e = plane ? (zp_e4(p, p->tune) || p->desc.prec == EQ_FP64 ? 4 : 8) : 0;
  return EQ_OK;
}

eq_status eq_plan_set_timing(eq_plan_t p, int enable) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  p->timing = enable != 0;
  return EQ_OK;
}

eq_status eq_plan_set_timing_pass(eq_plan_t p, const char* pass) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  if (!pass || !pass[0]) {
    p->timing_pass = -1;
    return EQ_OK;
  }
  for (int i = 0; i < P_COUNT; ++i)
    if (std::strcmp(kPassNames[i], pass) == 0) {
      p->timing_pass = i;
      return EQ_OK;
    }
  return fail(EQ_ERR_ARG, std::string("unknown pass ") + pass);
}

eq_status eq_plan_reset_stats(eq_plan_t p) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  DeviceGuard dg(p->device);
  EQ_HIP(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  for (auto& r : p->pending) { p->event_pool.push_back(r.a); p->event_pool.push_back(r.b); }
  p->pending.clear();
  for (int i = 0; i < P_COUNT; ++i) { p->launches[i] = 0; p->total_ms[i] = 0.0; p->total_bytes[i] = 0.0; }
  return EQ_OK;
}

eq_status eq_plan_pass_stats(eq_plan_t p, int max, int* count, const char** names, long long* launches,
                             double* total_ms, double* bytes_per_launch) {
  if (!p || !count) return fail(EQ_ERR_ARG, "null plan or count");
  DeviceGuard dg(p->device);
  if (!p->pending.empty()) {
    EQ_HIP(hipEventSynchronize(p->pending.back().b), "hipEventSynchronize");
    for (auto& r : p->pending) {
      float ms = 0.f;
      EQ_HIP(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
      p->total_ms[r.pass] += ms;
      p->launches[r.pass] += 1;
      p->event_pool.push_back(r.a);
      p->event_pool.push_back(r.b);
    }
    p->pending.clear();
  }
  *count = P_COUNT;
  for (int i = 0; i < P_COUNT && i < max; ++i) {
    if (names) names[i] = kPassNames[i];
    if (launches) launches[i] = p->launches[i];
    if (total_ms) total_ms[i] = p->total_ms[i];
    if (bytes_per_launch)
      bytes_per_launch[i] = p->launches[i] ? p->total_bytes[i] / (double)p->launches[i] : pass_bytes(p, i);
  }
  return EQ_OK;
}

eq_status eq_debug_forward(eq_plan_t p, const void* s_in, void* spec_out) {
  if (!p) return fail(EQ_ERR_ARG, "null plan");
  if (!s_in || !spec_out) return fail(EQ_ERR_ARG, "null pointer");
  DeviceGuard dg(p->device);
  auto go = [&](auto tag) -> eq_status {
    using T = decltype(tag);
    using C = cplx<T>;
    C* W = static_cast<C*>(spec_out);
    const C* tw = reinterpret_cast<const C*>(sizeof(T) == 8 ? (const void*)p->tw64 : (const void*)p->tw32);
    EQ_HIP(launch_z_r2c<T>(static_cast<const T*>(s_in), W, p->g, p->az, tw + p->g.nx + p->g.ny, p->tune, p->stream), "z_r2c");
    const int total = p->g.batch * p->g.nzh;
    EQ_HIP(launch_y<T>(W, p->g, 0, total, 6, p->ay, tw + p->g.nx, false, p->tune, p->stream), "y_fwd");
    EQ_HIP(launch_x<T>(W, p->g, 0, total, XM_FWD, p->ax, tw, p->sym, p->tune, p->stream), "x_fwd");
    return EQ_OK;
  };
  return p->desc.prec == EQ_FP64 ? go(double{}) : go(float{});
}

eq_status eq_debug_project_spectrum(eq_plan_t p, void* spec) {
  if (!p || !spec) return fail(EQ_ERR_ARG, "null pointer");
  DeviceGuard dg(p->device);
  auto go = [&](auto tag) -> eq_status {
    using T = decltype(tag);
    using C = cplx<T>;
    const C* tw = reinterpret_cast<const C*>(sizeof(T) == 8 ? (const void*)p->tw64 : (const void*)p->tw32);
    EQ_HIP(launch_x<T>(static_cast<C*>(spec), p->g, 0, p->g.batch * p->g.nzh, XM_PROJ, p->ax, tw, sym_unit(p), p->tune,
                       p->stream),
           "proj_only");
    return EQ_OK;
  };
  return p->desc.prec == EQ_FP64 ? go(double{}) : go(float{});
}

}  // extern "C"
