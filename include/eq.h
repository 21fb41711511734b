/*
 * eq.h -- C ABI of libeq: equilibrium projection of voxelized symmetric stress
 * fields on AMD Instinct MI355X (gfx950).
 *
 * The operation (Zhou, Lebensohn, Reischig, Ludwig, Bhattacharya, "Imposing
 * equilibrium on measured 3-D stress fields using Hodge decomposition and
 * FFT-based optimization"):
 *
 *   S_equil = argmin { ||S - S_exp||_2 : S periodic, symmetric, div S = 0 }
 *                                         (Section 3.2, problem statement)
 *
 * solved in Fourier space (Section 3.3 solution strategy, Section 4): the mean
 * c0 of S_exp is kept, and at every frequency q with a nonzero derivative
 * symbol s(q) the spectrum A(q) (a complex symmetric 3x3 matrix) is replaced by
 * curl H curl with nabla^4 H = curl A curl (eqnELH, eq:sequil), which equals
 * P A P with P = I - n n^T, n = s/|s|.  Frequencies whose symbol vanishes (the
 * mean and the 7 Nyquist corners of an even grid) are divergence-free under
 * the discrete operator and are kept unchanged.  The removed part
 * S_exp - S_equil is the symmetrized gradient of Theorem 2.
 *
 * Two derivative symbols (Section 4):
 *   EQ_OP_CDO  continuous:  xi(q) = 2 pi k(q) / (n h), k = q (q < n/2),
 *              0 (q = n/2), q - n (q > n/2)                      (eq:cdo)
 *   EQ_OP_DDO  central difference (the paper's operator for interfaces):
 *              s(q) = sin(2 pi q / n) / h                        (eq:diff)
 *
 * Data conventions (every entry point):
 *   - a field is C-contiguous (6, nz, ny, nx), x fastest; a batch is
 *     (batch, 6, nz, ny, nx); components in Voigt order (11, 22, 33, 23, 13, 12)
 *     with tensor index 1 = x, 2 = y, 3 = z;
 *   - element type is double (EQ_FP64) or float (EQ_FP32) per eq_desc.prec;
 *   - all field buffers are caller-owned DEVICE pointers on the plan's device;
 *     the library never frees or retains them beyond a call (except the
 *     graph cache of EQ_F_CAPTURE_GRAPH, which remembers their addresses);
 *   - the norm is Frobenius: off-diagonal Voigt components weigh 2.
 *
 * Errors: every call returns an eq_status; nothing aborts or throws across the
 * ABI.  eq_last_error() returns a thread-local message for the last failure.
 * Argument checks happen on the host before any device work is enqueued.
 */
#ifndef EQ_H
#define EQ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eq_plan_s* eq_plan_t;   /* opaque; from eq_plan, freed by eq_plan_destroy */

typedef enum {
  EQ_OK = 0,
  EQ_ERR_ARG = 1,        /* null/aliased pointer, bad enum, bad h, batch < 1, bad flags */
  EQ_ERR_SIZE = 2,       /* a grid edge is odd, < 4, > 1024, or has a prime factor > 5; or
                            nx / (largest of 8, 4, 2 dividing nx) > 170; or LDS beyond the device limit */
  EQ_ERR_NOMEM = 3,      /* device allocation failed (or EQ_FAULT_INJECT=alloc) */
  EQ_ERR_DEVICE = 4,     /* a HIP runtime call failed; see eq_last_error() */
  EQ_ERR_NONFINITE = 5   /* EQ_F_CHECK_FINITE: the input holds a NaN or Inf */
} eq_status;

typedef enum { EQ_OP_CDO = 0, EQ_OP_DDO = 1 } eq_op;
/* EQ_FP32: float data and FFT arithmetic; twiddles and symbols are generated in
 * FP64 on the device, and the per-frequency normalization 1/|s| is formed in FP64. */
typedef enum { EQ_FP64 = 0, EQ_FP32 = 1 } eq_prec;

enum {
  EQ_F_CHECK_FINITE = 1u,   /* eq_project scans the input and synchronizes; NaN/Inf -> EQ_ERR_NONFINITE */
  EQ_F_CAPTURE_GRAPH = 2u,  /* eq_project records its launches once per (s_in, s_eq, s_removed) and
                               replays a hipGraph afterwards; needs a stream other than the null stream */
  EQ_F_PERSISTENT = 4u,     /* eq_project runs as one launch for the whole batch: workgroups take work items
                               (forward xy planes, z columns, inverse planes) from a device-side queue in an
                               order that lets fields overlap, each field's stages ordered by per-field counters.
                               FP32 with nx == ny in {64, 128} and nz in {64, 128, 256} (else EQ_ERR_ARG at
                               eq_plan).  Its z stage runs four elements per thread, as the three-pass schedule
                               does with eq_tune zp_e = 4, whose results it equals bit for bit.  A counter wait
                               that gives up (never expected) is reported by eq_residual as
                               EQ_ERR_DEVICE, then and on every later call: the flag stays set, later
                               launches of the plan give up early, and the plan must be destroyed.
                               The environment variable EQ_PERSIST_SPIN_LIMIT (polls, default 262144)
                               lowers the limit, for tests of this path. */
  EQ_F_OWN_STREAM = 8u      /* the plan creates and owns a non-blocking stream; hip_stream is ignored */
};

typedef struct {
  int nx, ny, nz;      /* grid edges: even, 4..1024, prime factors in {2, 3, 5} (Section 4: N even) */
  int batch;           /* independent fields of identical shape, >= 1 */
  int op;              /* eq_op */
  int prec;            /* eq_prec */
  double h;            /* voxel spacing, finite and > 0; L = n h.  The projection itself does not
                          depend on h (only the direction of s matters); residual norms do. */
  unsigned flags;      /* EQ_F_* */
} eq_desc;

/* Create a plan: validates *d on the host, allocates the device workspace
 * (the Hermitian half spectrum, batch * 6 * (nz/2+1) * ny * nx complex values),
 * and launches the FP64 table kernel (twiddles, symbols) once.
 * hip_stream: the hipStream_t to enqueue on; NULL is HIP's null stream.  With
 * EQ_F_OWN_STREAM the plan creates its own non-blocking stream instead.
 * The plan binds to the device current at this call.  Not thread-safe: one
 * plan per thread at a time; distinct plans may run concurrently. */
eq_status eq_plan(const eq_desc* d, void* hip_stream, eq_plan_t* out);

/* Equilibrate: s_eq = S_equil(s_in); s_removed (nullable) = s_in - s_eq.
 * Buffers: device, (batch, 6, nz, ny, nx) of the plan's element type.
 * s_eq == s_in (in place) is allowed; s_removed must not overlap either.
 * Stream-ordered and asynchronous (except with EQ_F_CHECK_FINITE). */
eq_status eq_project(eq_plan_t p, const void* s_in, void* s_eq, void* s_removed);

/* Divergence residual r_i = sum_j D_j S_ij of a field under the plan's operator
 * (Section 5 divergence maps).  DDO uses real-space central differences (exactly
 * the DDO symbol); CDO uses the spectral symbol.  Accumulation in FP64.
 * norms_host: HOST array [batch][3] = { l2 = sqrt(sum_x |r|^2),
 *   max = max_x |r(x)|, rel = l2 / (max_q |s(q)| * ||s - mean(s)||_F) }.
 * div_out (nullable): DEVICE (batch, 3, nz, ny, nx) of the element type.
 * Blocks until norms_host is written. */
eq_status eq_residual(eq_plan_t p, const void* s, double* norms_host, void* div_out);

/* eq_residual without any allocation, for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid hipMalloc).
 * No plan: *d describes the fields (its flags are ignored) and the call enqueues the DDO
 * stencil and the final reduction on hip_stream (NULL = the null stream) of the current
 * device.  The per-workgroup partial sums live in a static device array of the library
 * (7.3 MB per device, held until the process ends), so at most 64 fields per call.
 *   d         : as for eq_plan; op must be EQ_OP_DDO (the CDO residual needs a plan's
 *               spectrum workspace) else EQ_ERR_ARG; batch > 64 -> EQ_ERR_SIZE;
 *   s         : device (batch, 6, nz, ny, nx), element type per d->prec;
 *   norms_dev : DEVICE double [batch][3] = { l2, max, rel } as eq_residual's norms_host;
 *   div_out   : nullable, DEVICE (batch, 3, nz, ny, nx) of the element type.
 * Stream-ordered and asynchronous (nothing is copied to the host).  Every call on one
 * device shares the array: calls that overlap in time on one device race, so serialize
 * them (one stream, or events).  Values equal eq_residual's to rounding of the final
 * division and square roots, which here run on the device. */
eq_status eq_residual_noalloc(const eq_desc* d, void* hip_stream, const void* s, double* norms_dev, void* div_out);

/* Non-periodic sample in a zero-stress lateral buffer (Section 3.3; Section 5.2, experimental
 * sample): the sample (nx0 x ny0 voxels in x and y, all nz planes, so top and bottom are
 * periodically connected) sits at (ox, oy) inside the plan's periodic (nx, ny) box; every
 * other voxel of the box is zero stress.  The box is projected as by eq_project and the
 * result is returned on the sample's voxels only.
 *   e     : 1 <= nx0, 0 <= ox, ox + nx0 <= nx (same for y), else EQ_ERR_ARG;
 *   s_in  : device (batch, 6, nz, ny0, nx0), the plan's precision;
 *   s_eq  : device, same shape (may equal s_in);
 *   s_removed : nullable, same shape, s_in - s_eq; must not overlap the others.
 * Always runs the five-pass schedule (the z passes read and write the sample in place of the
 * box, so no box-sized field is ever stored) and never replays a captured graph.
 * Stream-ordered and asynchronous. */
typedef struct { int nx0, ny0, ox, oy; } eq_embed;
eq_status eq_project_embedded(eq_plan_t p, const eq_embed* e, const void* s_in, void* s_eq, void* s_removed);

/* Potential of the removed part (Section 3.2: S_exp = S_equil + (grad y + grad y^T)/2).
 * Writes the periodic vector field y whose symmetric gradient, in the plan's operator
 * (CDO or DDO, with spacing h), is exactly S_exp - S_equil: per frequency
 * y = i (c n - 2 b) / |s| with n = s/|s|, b = A n, c = n.b, and y = 0 where the symbol is
 * zero (so y has zero mean; the harmonic modes belong to S_equil).
 *   s_in  : device (batch, 6, nz, ny, nx), the plan's precision (not modified);
 *   y_out : device (batch, 3, nz, ny, nx), components (y_x, y_y, y_z), caller-owned;
 *           must not overlap s_in (EQ_ERR_ARG).
 * Uses the plan workspace (five-pass kernels); stream-ordered and asynchronous.  With
 * EQ_F_CHECK_FINITE, synchronizes and returns EQ_ERR_NONFINITE on NaN/Inf input. */
eq_status eq_potential(eq_plan_t p, const void* s_in, void* y_out);

eq_status eq_plan_destroy(eq_plan_t p);

/* Device bytes a plan for *d allocates (workspace + tables + reduction scratch),
 * for admission control; host only, no device call. */
eq_status eq_plan_footprint(const eq_desc* d, size_t* bytes);

const char* eq_status_str(eq_status s);
const char* eq_last_error(void);

/* Rebind the plan to another stream (NULL = the null stream); drops cached graphs. */
eq_status eq_plan_set_stream(eq_plan_t p, void* hip_stream);

/* Per-pass instrumentation.  When enabled, every kernel of eq_project/eq_residual is
 * bracketed by hipEvents on the plan stream; eq_plan_pass_stats synchronizes and
 * reports, per pass i < *count: name, launches, summed milliseconds and the
 * algorithmic bytes (compulsory reads + writes) of one launch.  Graph replay is
 * bypassed while enabled. */
eq_status eq_plan_set_timing(eq_plan_t p, int enable);
/* Restrict the instrumentation to the pass named `pass` (a name eq_plan_pass_stats
 * reports, e.g. "z_c2r"); NULL or "" = every pass.  Each bracketed launch adds two event
 * records to the stream, so timing one pass keeps the instrumented step close to the
 * uninstrumented one.  Unknown names return EQ_ERR_ARG.  Timing itself is still switched
 * by eq_plan_set_timing. */
eq_status eq_plan_set_timing_pass(eq_plan_t p, const char* pass);
eq_status eq_plan_pass_stats(eq_plan_t p, int max, int* count, const char** names,
                             long long* launches, double* total_ms, double* bytes_per_launch);
eq_status eq_plan_reset_stats(eq_plan_t p);

/* Launch-shape and radix-schedule tuning (the autotuner's knobs; 0 = library default for
 * the shape knobs, -1 for radix16):
 *   tx_y     x-columns per workgroup of the y passes (must divide nx),
 *   tx_z     real x-columns per workgroup of the z passes (even, must divide nx),
 *   rw_x     (kz, ky) rows per workgroup of the fused x pass,
 *   chunk    planes (field, kz) per chunk of the y -> x -> y sequence, so that a chunk's
 *            spectrum can stay in the last-level cache between passes (0 or -1: one chunk),
 *   radix16  bit mask of the axes (1 = x, 2 = y, 4 = z) whose power-of-two edges >= 128 use
 *            radix-16 stages instead of radix-8 ones; -1 = library default (y only),
 *   schedule pass schedule of eq_project: 5 = five passes (z, y, x + projection, y, z);
 *            3 = three passes (xy plane, z + projection, xy plane), available when
 *            nx == ny in {64, 128, 256} (FP64: 64, 128) and nz in {64, 128, 256};
 *            0 = library default (three passes where available and nx <= 128),
 *   tc_zp    (ky, kx) columns per workgroup of the three-pass z projection (must divide ny),
 *   radix4   1: radix-4 stages on x (FP32): nx a power of two in 32 .. 512 (the six-component
 *            x kernel then holds 6 x 4 values per lane instead of 6 x 8), or nx 96, 160, 192,
 *            320 or 384 with the split x kernel (xsplit 0 or 2; E = 12 or 20 instead of 24 or
 *            40); ignored elsewhere and with xsplit = 1 on those edges,
 *   xsplit   x pass kernel: 2 = six components split over the two halves of a wavefront
 *            (three rows of E values per lane; needs nx / E to divide 32), 1 = not split,
 *            0 = library default; reported as 1 or 2,
 *   zp_e     elements per thread of the three-pass z projection in FP32: 8 (default) or 4
 *            (half the registers per thread, radix-4 stages); 0 = default; FP64 always uses 4;
 *            reported as 4 or 8 on the three-pass route (4 under EQ_F_PERSISTENT), else 0.
 * Invalid shapes for this grid return EQ_ERR_ARG (EQ_ERR_SIZE if LDS would exceed the device
 * limit) and leave the plan unchanged.  Every setting computes the same transform; results
 * may differ only by floating-point rounding order (radix16, radix4, zp_e and schedule change
 * the radix stages or the pass order; the other knobs can change which kernel serves a pass).
 * The EQ_TUNE environment variable ("tx_y=16,tx_z=32,rw_x=4,chunk=32,radix16=2,schedule=5") seeds the
 * tuning at eq_plan.  eq_plan_get_tune reports the settings in effect (defaults resolved). */
typedef struct { int tx_y, tx_z, rw_x, chunk, radix16, schedule, tc_zp, radix4, xsplit, zp_e; } eq_tune;
eq_status eq_plan_tune(eq_plan_t p, const eq_tune* t);
eq_status eq_plan_get_tune(eq_plan_t p, eq_tune* t);

/* Test hooks (same kernels as eq_project, exposed for per-stage parity):
 * eq_debug_forward: spec_out (device) = the unnormalized forward DFT of s_in as
 *   complex (re, im) pairs laid out (batch, 6, nz/2+1, ny, nx) -- the half spectrum
 *   along z, full along y and x.
 * eq_debug_project_spectrum: in place on such a half spectrum, apply the
 *   per-frequency projection (forward and inverse x transforms around it are
 *   skipped). */
eq_status eq_debug_forward(eq_plan_t p, const void* s_in, void* spec_out);
eq_status eq_debug_project_spectrum(eq_plan_t p, void* spec_inout);

/* Library build string. */
const char* eq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EQ_H */
