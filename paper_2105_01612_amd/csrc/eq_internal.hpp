// eq_internal.hpp -- host-side interface between the plan (eq_capi.cpp) and the
// kernel launchers (eq_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

#include "eq_fft.hpp"

namespace eq {

// Grid geometry of one plan.  The spectrum workspace W holds, per field, the
// Hermitian half along z: (batch, 6, nzh = nz/2 + 1, ny, nx) complex.
// A "plane" is one (field, kz) pair, pl = b * nzh + kz; the y and x passes take
// a contiguous plane range so the plan can run them chunk by chunk.
struct Geom {
  int nx, ny, nz, nzh, batch;
};

struct AxisFft {
  FftDesc d;   // radix schedule of this axis
  int E;       // elements per thread: 8/16/24/40 (register engine) or 2/4/8 (generic engine)
  bool fast;   // register engine (every radix divides E)
};

// Launch shape knobs (0 = library default).  The autotuner may set them.
struct Tune {
  int tx_y = 0;    // x-tile width of the y pass (lines per workgroup)
  int tx_z = 0;    // x-tile width of the z passes (real columns per workgroup, even)
  int rw_x = 0;    // rows per workgroup of the fused x pass
  int chunk = 0;   // planes per chunk of the y/x/y sequence (0 = library default, -1 = no chunking)
  int radix16 = -1;  // axes (1 = x, 2 = y, 4 = z) using radix-16 schedules; -1 = default (y)
  int schedule = 0;  // 5 = five passes, 3 = three passes (plane route), 0 = default
  int tc_zp = 0;     // columns per workgroup of the three-pass z projection
  int radix4 = 0;    // 1: radix-4 stages on x (six-component x kernel, FP32 powers of two)
  int xsplit = 0;    // six-component x kernel split over wavefront halves: 1 = off, 2 = on, 0 = default
  int zp_e = 0;      // elements per thread of the three-pass z projection in FP32: 8 or 4 (0 = default 8)
};

// Lateral embedding of a sample in the periodic box (the zero-stress buffer of Sections 3.3
// and 6): the real field that the z passes read and write is (.., nz, ny0, nx0), placed at
// (ox, oy) in the (ny, nx) plane of the box.  Box voxels outside the sample read as zero and
// are not written.  on = false: the real field is the whole box.
struct Embed {
  int nx0 = 0, ny0 = 0, ox = 0, oy = 0;
  bool on = false;
};

// Modes of the fused x pass.
enum XMode : int {
  XM_FWD = 1,        // forward DFT along x
  XM_PROJ = 2,       // per-frequency projection P A P
  XM_INV = 4,        // inverse DFT along x
  XM_DIV = 8,        // per-frequency divergence i s_j A_ij -> components 0..2
  XM_DISP = 16,      // per-frequency potential of the removed part -> components 0..2
};

// Symbol table layout: sym[0 .. nx) x-axis, sym[nx .. nx+ny) y, sym[nx+ny .. +nz) z.
// Twiddle tables: tw[off_a + m] = exp(-2 pi i m / n_a) with off_x = 0, off_y = nx, off_z = nx + ny.

hipError_t launch_tables(const Geom& g, int op, double h, double* sym, double2* tw64, float2* tw32,
                         hipStream_t s);

template <typename T>
hipError_t launch_z_r2c(const T* in, cplx<T>* W, const Geom& g, const AxisFft& az, const cplx<T>* tw_z,
                        const Tune& tn, hipStream_t s, const Embed& e = Embed{});

template <typename T>
hipError_t launch_y(cplx<T>* W, const Geom& g, int pl0, int npl, int ncomp, const AxisFft& ay, const cplx<T>* tw_y,
                    bool inv, const Tune& tn, hipStream_t s);

// h: voxel spacing, used by XM_DISP only (its symbols are h-free)
template <typename T>
hipError_t launch_x(cplx<T>* W, const Geom& g, int pl0, int npl, int mode, const AxisFft& ax, const cplx<T>* tw_x,
                    const double* sym, const Tune& tn, hipStream_t s, double h = 1.0);

// out(b, c, z, y, x) = out + b * out_field + c * out_comp + (z * ny + y) * nx + x for c < ncomp
// (with an embedding: sample coordinates, (z * ny0 + y - oy) * nx0 + x - ox, sample voxels only).
// removed (nullable) = in - out at the same offsets.
template <typename T>
hipError_t launch_z_c2r(const cplx<T>* W, T* out, size_t out_field, size_t out_comp, const T* in, T* removed,
                        int ncomp, const Geom& g, const AxisFft& az, const cplx<T>* tw_z, const Tune& tn,
                        hipStream_t s, const Embed& e = Embed{});

// Reduction record per field (kRedWidth doubles):
//   [0] sum_x |r|^2, [1] max_x |r|^2, [2..7] sum_x d_c, [8..13] sum_x d_c^2 with d_c = S_c - S_c(first voxel)
constexpr int kRedWidth = 14;

// DDO residual; nblk_max bounds the workgroups per field (partials holds batch * nblk_max
// records).  div_ddo_blocks returns how many it uses, for the final reduction.
template <typename T>
hipError_t launch_div_ddo(const T* S, T* div_out, double* partials, int nblk_max, const Geom& g, double h,
                          hipStream_t s);
int div_ddo_blocks(const Geom& g, int nblk_max, bool fp64);

template <typename T>
hipError_t launch_div_stats(const T* div, size_t div_field, size_t div_comp, const T* S, double* partials,
                            int nblk, const Geom& g, hipStream_t s);

hipError_t launch_reduce_final(const double* partials, int nblk, int batch, double* out, hipStream_t s);

// Partial records per field (an upper bound on the residual's workgroups per field).
constexpr int kRedBlocks = 1024;
// Allocation-free residual: at most kNoAllocFields fields per call; its partial records live
// in a static device array whose address noalloc_scratch returns for the current device.
constexpr int kNoAllocFields = 64;
hipError_t noalloc_scratch(double** out);
// The final reduction finished on the device: norms[b] = (l2, max, rel), inv_m = 1 / voxels
// per field, smax = max_q |s(q)|.
hipError_t launch_reduce_norms(const double* partials, int nblk, int batch, double inv_m, double smax, double* norms,
                               hipStream_t s);

template <typename T>
hipError_t launch_check_finite(const T* in, size_t n, int* flag, hipStream_t s);

hipError_t launch_fill_int(int* p, int n, int value, hipStream_t s);

// Three-pass schedule (eq_plane.hip).  Spectrum workspace W2 = (batch, 6, nz, ny, nx/2 + 1)
// complex; a plane is (field, component, z).
bool plane_route_supported(const Geom& g, bool fp64);
size_t plane_lds(const Geom& g, bool fp64);
int pick_tc_zproj(const Geom& g, bool fp64, int want, bool e4);
size_t zproj_lds(const Geom& g, bool fp64, int tc);

template <typename T>
hipError_t launch_plane_r2c(const T* in, cplx<T>* W2, const Geom& g, const cplx<T>* twx, const cplx<T>* twy,
                            hipStream_t s);
template <typename T>
// e4: four elements per thread along z (FP32; FP64 always takes four)
hipError_t launch_zproj(cplx<T>* W2, const Geom& g, const cplx<T>* twz, const double* symu, int tc, bool e4,
                        hipStream_t s);
// out, removed (nullable): field layout; removed = in - out
template <typename T>
hipError_t launch_plane_c2r(const cplx<T>* W2, T* out, const T* in, T* removed, const Geom& g, const cplx<T>* twx,
                            const cplx<T>* twy, hipStream_t s);

// Persistent three-pass launch (EQ_F_PERSISTENT, FP32): nx == ny in {64, 128}, nz in {64, 128,
// 256}.  ctr: 4 + 2 * batch counters, zero before the first launch (each launch leaves them zero,
// except ctr[2], raised if a dependency wait gave up).
bool persist_route_supported(const Geom& g, bool fp64);
template <typename T>
hipError_t launch_persist(const T* in, cplx<T>* W2, T* out, T* removed, const Geom& g, const cplx<T>* twx,
                          const cplx<T>* twy, const cplx<T>* twz, const double* symu, unsigned* ctr, hipStream_t s);

// Launch shapes (exposed so the plan can check LDS against the device limit).
int pick_tx_y(const Geom& g, const AxisFft& ay, int elem_bytes, const Tune& tn);
int pick_tx_z(const Geom& g, const AxisFft& az, int elem_bytes, const Tune& tn);
int pick_rw_x(const Geom& g, const AxisFft& ax, int elem_bytes, const Tune& tn);
int max_threads(const AxisFft& ax);
int x_threads_per_row(const AxisFft& ax, int elem_bytes, const Tune& tn);   // threads of the x pass per (kz, ky) row
bool x6_radix4_available(int nx, bool fp64);   // radix-4 x schedules exist only for the six-component kernels
bool x_split(const AxisFft& ax, int elem_bytes, const Tune& tn);   // x pass takes the half-split kernel
size_t lds_y(const Geom& g, const AxisFft& ay, int elem_bytes, const Tune& tn);
size_t lds_z(const Geom& g, const AxisFft& az, int elem_bytes, const Tune& tn);
size_t lds_x(const Geom& g, const AxisFft& ax, int elem_bytes, const Tune& tn);

}  // namespace eq
