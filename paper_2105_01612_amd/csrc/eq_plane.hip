// eq_plane.hip -- three-pass schedule of the projection for grids whose xy plane of
// one component fits one workgroup (registers + LDS):
//
//   plane_r2c : per (field, component, z) plane: real-to-complex DFT along x, complex
//               DFT along y  ->  W2(b, c, z, ky, kx) for kx in [0, nx/2), and the Nyquist
//               column kx = nx/2 in its own array W2N(b, c, z, ky) after W2, so that
//               every row of W2 is a whole number of 128-byte lines
//   zproj     : per (ky, kx) column: DFT along z of all six components, projection
//               P A P per frequency in registers, inverse DFT along z
//   plane_c2r : per plane: inverse DFT along y, complex-to-real along x, 1/N scaling,
//               removed = in - out
//
// Each pass reads and writes the field or its half spectrum once, so the projection
// moves three round trips of HBM instead of five.  The forward and inverse DFTs are
// the unnormalized analysis/synthesis pair of Section 4 (eqnFFT/eqniFFT, with the
// 1/N^3 on the synthesis side); the per-frequency projection is Theorem 2 in the
// P A P form (Section 3.2, eq:sequil with the gauge of eqnELH).
//
// Real-to-complex along x packs rows 2j and 2j+1 of a plane into one complex line,
// z = a + i b, and separates the two half spectra from Z(k) and Z(n - k).  Columns
// kx = 0 and kx = nx/2 of the x spectrum hold real values per row; they travel
// through the y DFT packed as one complex column (DC + i Nyquist) and are separated
// the same way.  The inverse path undoes both packings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "eq_fft.hpp"
#include "eq_internal.hpp"
#include "eq_persist_queue.hpp"
#include "eq_kernels_impl.hpp"

namespace eq {
namespace {

// Thread maps.  x phase: thread (px, lx) owns elements x = px + i*PX of packed lines
// j = lx + r*LX (r < RX); its x DFT leaves Z_j(k), k = px + i*PX, in registers.  y phase:
// round ry handles half-spectrum columns kx in [ry*LY, ry*LY + LY); thread (cy, py) owns
// rows y = py + i*PY of column kx = ry*LY + cy.  Between the two, a round's columns pass
// through an LDS tile (ZA: Z_j(kx), ZB: Z_j(nx - kx), with ZB at kx = 0 holding the
// Nyquist Z_j(nx/2)); the inverse kernel runs the same maps backwards with a tile of
// real-row spectra.
template <typename T, int NX, int NY, int NT, typename FX, typename FY>
struct PlaneShape {
  static constexpr int EX = FX::E, PX = NX / EX, LX = NT / PX, RX = (NY / 2) / LX;
  static constexpr int EY = FY::E, PY = NY / EY, LY = NT / PY, RY = (NX / 2) / LY;
  static constexpr int NXH = NX / 2, NJ = NY / 2;          // W2 row length (Nyquist apart)
  static constexpr int LSX = NX + (NX >> kSkew) + 1;  // LDS stride of one x line (skewed)
  static constexpr int TS = LY + 1;                  // LDS stride of one tile row
  // forward: ZA, ZB (NJ rows each), y exchange (LY columns), column-0 buffer (NY);
  // inverse: tile of NY rows, y exchange.  The x exchange overlaps either.
  static constexpr int YOFF = 2 * NJ * TS;
  static constexpr int COFF = YOFF + NY * LY;
  static constexpr int lds_fwd = COFF + NY;
  static constexpr size_t lds_elems = (size_t)(LX * LSX > lds_fwd ? LX * LSX : lds_fwd);
  static_assert(FX::N == NX && FY::N == NY, "schedule length");
  static_assert(LX * PX == NT && RX * LX == NY / 2, "x phase must tile the plane");
  static_assert(LY * PY == NT && RY * LY == NX / 2, "y phase must tile the half spectrum");
  static_assert(PY % 2 == 0, "rows 2j and 2j+1 of one y-column belong to neighbouring threads");
};

// Forward plane `plane` of `planes` (one workgroup; LDS of PlaneShape::lds_elems at `lds`).
template <typename T, int NX, int NY, int NT, typename FX, typename FY>
__device__ __forceinline__ void plane_r2c_body(const T* __restrict__ in, cplx<T>* __restrict__ W2, int plane,
                                               int planes, const cplx<T>* __restrict__ twx,
                                               const cplx<T>* __restrict__ twy, cplx<T>* lds, int tid) {
  using C = cplx<T>;
  using S = PlaneShape<T, NX, NY, NT, FX, FY>;
  constexpr int EX = S::EX, PX = S::PX, LX = S::LX, RX = S::RX;
  constexpr int EY = S::EY, PY = S::PY, LY = S::LY, RY = S::RY, NXH = S::NXH, TS = S::TS;
  C* ZA = lds;
  C* ZB = lds + S::NJ * TS;
  C* YX = lds + S::YOFF;
  C* CB = lds + S::COFF;
  const FftDesc dd{};
  const T* src = in + (size_t)plane * (NX * NY);
  C* dst = W2 + (size_t)plane * (NXH * NY);
  C* dstn = W2 + (size_t)planes * (NXH * NY) + (size_t)plane * NY;   // Nyquist column
  const int px = tid % PX, lx = tid / PX;
  // ---- x phase: packed line j = lx + r*LX holds rows 2j (real part) and 2j+1 (imaginary part)
  C v[RX][EX];
  const LdsMap mx{S::LSX, 1, kSkew};
#pragma unroll
  for (int r = 0; r < RX; ++r) {
    const T* row = src + (size_t)(2 * (lx + r * LX)) * NX + px;
#pragma unroll
    for (int i = 0; i < EX; ++i) v[r][i] = mk<T>(row[i * PX], row[NX + i * PX]);
    FX::template run<T, 1, false, true, true>(&v[r], lds, mx, lx, 0, px, dd, twx);
    __syncthreads();
  }
  // ---- y phase
  const int cy = tid % LY, py = tid / LY;
  const LdsMap my{1, LY, 0};
  const T half = (T)0.5;
#pragma unroll
  for (int ry = 0; ry < RY; ++ry) {
    const int c0 = ry * LY;
#pragma unroll
    for (int r = 0; r < RX; ++r)
#pragma unroll
      for (int i = 0; i < EX; ++i) {
        // addresses stay affine in (px, lx) per (r, i): one base register serves every store
        const int k = px + i * PX, j = lx + r * LX;
        if (k >= c0 && k < c0 + LY) ZA[j * TS + k - c0] = v[r][i];
        if (i == NX / (2 * PX) && px == 0) {
          if (c0 == 0) ZB[j * TS] = v[r][i];               // Nyquist Z_j(nx/2) rides in column 0
        } else if (NX - k >= c0 && NX - k < c0 + LY) {
          ZB[j * TS + (NX - k) - c0] = v[r][i];             // k = 0 gives nx - k = nx: never stored
        }
      }
    __syncthreads();
    const int kx = c0 + cy;
    C u[1][EY];
#pragma unroll
    for (int i = 0; i < EY; ++i) {
      const int y = py + i * PY;
      const C Z = ZA[(y >> 1) * TS + cy], Zm = ZB[(y >> 1) * TS + cy];
      if (kx == 0) {
        // DC and Nyquist of a real row are real: carry them as (DC, Nyquist)
        u[0][i] = (y & 1) ? mk<T>(Z.y, Zm.y) : mk<T>(Z.x, Zm.x);
      } else {
        u[0][i] = (y & 1) ? mk<T>((Z.y + Zm.y) * half, (Zm.x - Z.x) * half)
                          : mk<T>((Z.x + Zm.x) * half, (Z.y - Zm.y) * half);
      }
    }
    FY::template run<T, 1, false, true, true>(u, YX, my, cy, 0, py, dd, twy);
    if (kx != 0) {
#pragma unroll
      for (int i = 0; i < EY; ++i) dst[(size_t)(py + i * PY) * NXH + kx] = u[0][i];
    }
    if (ry == 0) {
      // column 0 carries DC + i Nyquist: separate the two (Hermitian) spectra
      if (kx == 0) {
#pragma unroll
        for (int i = 0; i < EY; ++i) CB[py + i * PY] = u[0][i];
      }
      __syncthreads();
      if (kx == 0) {
#pragma unroll
        for (int i = 0; i < EY; ++i) {
          const int ky = py + i * PY;
          const C Y = u[0][i], Ym = CB[ky == 0 ? 0 : NY - ky];
          dst[(size_t)ky * NXH] = mk<T>((Y.x + Ym.x) * half, (Y.y - Ym.y) * half);
          dstn[ky] = mk<T>((Y.y + Ym.y) * half, (Ym.x - Y.x) * half);
        }
      }
    }
  }
}

template <typename T, int NX, int NY, int NT, typename FX, typename FY>
__global__ __launch_bounds__(NT) void k_plane_r2c(const T* __restrict__ in, cplx<T>* __restrict__ W2,
                                                  const cplx<T>* __restrict__ twx, const cplx<T>* __restrict__ twy) {
  extern __shared__ unsigned char smem_raw[];
  plane_r2c_body<T, NX, NY, NT, FX, FY>(in, W2, blockIdx.x, gridDim.x, twx, twy, reinterpret_cast<cplx<T>*>(smem_raw),
                                        threadIdx.x);
}

// Inverse plane `plane` of `planes`.  out may be in (in place): each thread reads the input
// values it overwrites, and no others, so out, in and removed carry no __restrict__.
template <typename T, int NX, int NY, int NT, typename FX, typename FY>
__device__ __forceinline__ void plane_c2r_body(const cplx<T>* __restrict__ W2, T* out, const T* in, T* removed,
                                               int plane, int planes, const cplx<T>* __restrict__ twx,
                                               const cplx<T>* __restrict__ twy, T scale, cplx<T>* lds, int tid) {
  using C = cplx<T>;
  using S = PlaneShape<T, NX, NY, NT, FX, FY>;
  constexpr int EX = S::EX, PX = S::PX, LX = S::LX, RX = S::RX;
  constexpr int EY = S::EY, PY = S::PY, LY = S::LY, RY = S::RY, NXH = S::NXH, TS = S::TS;
  C* TT = lds;                     // NY rows x LY columns of the round's real-row spectra
  C* YX = lds + S::YOFF;
  const FftDesc dd{};
  const C* src = W2 + (size_t)plane * (NXH * NY);
  const C* srcn = W2 + (size_t)planes * (NXH * NY) + (size_t)plane * NY;   // Nyquist column
  const size_t obase = (size_t)plane * (NX * NY);
  const int px = tid % PX, lx = tid / PX;
  const int cy = tid % LY, py = tid / LY;
  const LdsMap my{1, LY, 0};
  C v[RX][EX];
  // ---- y phase (inverse): column 0 packs the DC and Nyquist columns as DC + i Nyquist
#pragma unroll
  for (int ry = 0; ry < RY; ++ry) {
    const int c0 = ry * LY, kx = c0 + cy;
    C u[1][EY];
#pragma unroll
    for (int i = 0; i < EY; ++i) {
      const int ky = py + i * PY;
      const C* s = src + (size_t)ky * NXH;
      if (kx == 0) {
        C F0 = s[0], FN = srcn[ky];
        if (ky == 0 || 2 * ky == NY) { F0.y = (T)0; FN.y = (T)0; }   // self-conjugate rows are real
        u[0][i] = mk<T>(F0.x - FN.y, F0.y + FN.x);
      } else {
        u[0][i] = s[kx];
      }
    }
    FY::template run<T, 1, true, true, true>(u, YX, my, cy, 0, py, dd, twy);
#pragma unroll
    for (int i = 0; i < EY; ++i) TT[(py + i * PY) * TS + cy] = u[0][i];
    __syncthreads();
    // x owners gather Z_j(k) = A(k) + i B(k) (rows 2j, 2j+1) for their k in this round
#pragma unroll
    for (int r = 0; r < RX; ++r)
#pragma unroll
      for (int i = 0; i < EX; ++i) {
        // column holding k: k itself below nx/2, nx - k above, column 0 for the Nyquist;
        // which case applies is fixed by i except for px == 0 at i*PX == nx/2
        const int k = px + i * PX, j = lx + r * LX;
        const C* t0 = TT + (2 * j) * TS - c0;
        const C* t1 = t0 + TS;
        if (2 * i * PX < NX) {
          if (k >= c0 && k < c0 + LY) {
            const C A = t0[k], B = t1[k];
            v[r][i] = (k == 0) ? mk<T>(A.x, B.x) : mk<T>(A.x - B.y, A.y + B.x);
          }
        } else if (2 * i * PX == NX && px == 0) {
          if (c0 == 0) {
            const C A = t0[0], B = t1[0];
            v[r][i] = mk<T>(A.y, B.y);
          }
        } else if (NX - k >= c0 && NX - k < c0 + LY) {
          const C A = t0[NX - k], B = t1[NX - k];
          v[r][i] = mk<T>(A.x + B.y, B.x - A.y);
        }
      }
    __syncthreads();
  }
  // ---- x phase (inverse): real part -> row 2j, imaginary part -> row 2j+1
  const LdsMap mx{S::LSX, 1, kSkew};
#pragma unroll
  for (int r = 0; r < RX; ++r) {
    FX::template run<T, 1, true, true, true>(&v[r], lds, mx, lx, 0, px, dd, twx);
    const size_t row = obase + (size_t)(2 * (lx + r * LX)) * NX + px;
    if (removed) {
      T a[EX], b[EX];
#pragma unroll
      for (int i = 0; i < EX; ++i) { a[i] = in[row + i * PX]; b[i] = in[row + NX + i * PX]; }
#pragma unroll
      for (int i = 0; i < EX; ++i) {
        const T o0 = v[r][i].x * scale, o1 = v[r][i].y * scale;
        out[row + i * PX] = o0;
        out[row + NX + i * PX] = o1;
        removed[row + i * PX] = a[i] - o0;
        removed[row + NX + i * PX] = b[i] - o1;
      }
    } else {
#pragma unroll
      for (int i = 0; i < EX; ++i) {
        out[row + i * PX] = v[r][i].x * scale;
        out[row + NX + i * PX] = v[r][i].y * scale;
      }
    }
    __syncthreads();
  }
}

template <typename T, int NX, int NY, int NT, typename FX, typename FY>
__global__ __launch_bounds__(NT) void k_plane_c2r(const cplx<T>* __restrict__ W2, T* out, const T* in, T* removed,
                                                  const cplx<T>* __restrict__ twx, const cplx<T>* __restrict__ twy,
                                                  T scale) {
  extern __shared__ unsigned char smem_raw[];
  plane_c2r_body<T, NX, NY, NT, FX, FY>(W2, out, in, removed, blockIdx.x, gridDim.x, twx, twy, scale,
                                        reinterpret_cast<cplx<T>*>(smem_raw), threadIdx.x);
}

// ------------------------------------------------------------ z pass -------

// Raw buffer access (resource word 3 in eq_kernels_impl.hpp); the range in the resource
// is the field's byte size.
template <typename T>
__device__ __forceinline__ cplx<T> buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  cplx<T> v;
  if constexpr (sizeof(T) == 4) {
    const auto raw = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    __builtin_memcpy(&v, &raw, sizeof(v));
  } else {
    const auto raw = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    __builtin_memcpy(&v, &raw, sizeof(v));
  }
  return v;
}

template <typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, cplx<T> v) {
  if constexpr (sizeof(T) == 4) {
    decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) raw;
    __builtin_memcpy(&raw, &v, sizeof(v));
    __builtin_amdgcn_raw_buffer_store_b64(raw, r, voff, soff, 0);
  } else {
    decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0)) raw;
    __builtin_memcpy(&raw, &v, sizeof(v));
    __builtin_amdgcn_raw_buffer_store_b128(raw, r, voff, soff, 0);
  }
}

struct ZpArgs {
  int nx, ny, nz, tc;        // tc: columns per workgroup (divides ny)
  int batch;
};

// Thread (col, p) owns elements kz = p + i*P of the six component columns of one
// (ky, kx); the forward DFTs, the projection and the inverse DFTs run in registers,
// with the LDS exchanges of consecutive transforms alternating between two regions.
// Z tiles of a field: ny * nx/2 / tc over W2 (kx < nx/2), then ny / tc over the Nyquist columns.
__host__ __device__ __forceinline__ int zproj_tiles(const ZpArgs& a) { return a.ny * (a.nx / 2) / a.tc + a.ny / a.tc; }

// Tile `tile` of field `b` (one workgroup of tc * NZ / E threads).
template <typename T, typename FZ>
__device__ __forceinline__ void zproj_body(cplx<T>* __restrict__ W2, const ZpArgs& a, const cplx<T>* __restrict__ tw,
                                           const double* __restrict__ sym, int tile, int b, cplx<T>* lds, int tid) {
  using C = cplx<T>;
  constexpr int E = FZ::E, NZ = FZ::N, P = NZ / E;
  const FftDesc dd{};
  // columns: ny * nx/2 of W2 (kx < nx/2), then ny Nyquist columns of W2N; a tile lies
  // wholly in one of the two, so its base and column stride are workgroup-uniform
  const int half = a.nx / 2;
  const int ntm = a.ny * half / a.tc;
  const int col = tid % a.tc, p = tid / a.tc;
  const bool nyq = tile >= ntm;
  const int plane = nyq ? a.ny : a.ny * half;
  const int f = (nyq ? tile - ntm : tile) * a.tc + col;
  const int ky = nyq ? f : f / half, kx = nyq ? half : f - (f / half) * half;
  C* region = nyq ? W2 + (size_t)a.batch * 6 * NZ * a.ny * half : W2;
  // element (c, kz = p + i*P) sits at this thread's byte offset (a VGPR) plus a
  // workgroup-uniform offset for (c, i) (an SGPR): buffer instructions take both, so
  // the 6*E addresses cost no registers of their own
  const unsigned fbytes = (unsigned)(6 * NZ) * (unsigned)plane * (unsigned)sizeof(C);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(region + (size_t)b * 6 * NZ * plane, 0, fbytes, kBufWord3);
  const unsigned voff = (unsigned)(f + p * plane) * (unsigned)sizeof(C);
  auto soff = [&](int c, int i) -> unsigned { return (unsigned)((c * NZ + i * P) * plane) * (unsigned)sizeof(C); };
  C v[6][E];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int i = 0; i < E; ++i) v[c][i] = buf_load<T>(rs, voff, soff(c, i));
  constexpr int LS = NZ + (NZ >> kSkew) + 1;   // contiguous, skewed column lines: stage offsets fold into immediates
  const LdsMap m{LS, 1, kSkew};
  C* reg[2] = {lds, lds + (size_t)a.tc * LS};
#pragma unroll
  for (int c = 0; c < 6; ++c) FZ::template run<T, 1, false, true, true>(&v[c], reg[c & 1], m, col, 0, p, dd, tw);
  const double sx = sym[kx], sy = sym[a.nx + ky];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    C A[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) A[c] = v[c][i];
    project_one<T>(A, sx, sy, sym[a.nx + a.ny + p + i * P]);
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c][i] = A[c];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) FZ::template run<T, 1, true, true, true>(&v[c], reg[c & 1], m, col, 0, p, dd, tw);
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int i = 0; i < E; ++i) buf_store<T>(rs, voff, soff(c, i), v[c][i]);
}

template <typename T, typename FZ>
__global__ __launch_bounds__(kMaxFastThreads) void k_zproj(cplx<T>* __restrict__ W2, ZpArgs a,
                                                           const cplx<T>* __restrict__ tw,
                                                           const double* __restrict__ sym) {
  extern __shared__ unsigned char smem_raw[];
  // workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous range of
  // tiles so that neighbouring narrow tiles share the 128-byte lines of their L2
  int bid = blockIdx.x;
  if ((gridDim.x & 7) == 0) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  const int ntile = zproj_tiles(a);
  zproj_body<T, FZ>(W2, a, tw, sym, bid % ntile, bid / ntile, reinterpret_cast<cplx<T>*>(smem_raw), threadIdx.x);
}

// ---------------------------------------------------------- persistent -----

// One launch runs the three passes of a whole batch.  Workgroups claim work items in queue
// order from a device-side counter.  Queue step s holds the forward planes of field s, the z
// tiles of field s - L and the inverse planes of field s - 2L (L >= 1, the lag: enough steps
// that the items a wait depends on have mostly finished when it is claimed, with a whole grid
// of workgroups in flight), so an item only ever waits for items earlier in the queue (claimed
// by workgroups that are running), and stages of different fields overlap.  A z item of field b starts once every forward item of b is done,
// an inverse item once every z item of b is done: per-field counters, raised after an item's
// stores are complete and written back (agent-scope release), read before the item's loads
// (agent-scope acquire).  Each item runs the same code as its pass kernel, so results are
// bitwise those of the three launches; no output is written by an atomic.
constexpr size_t kPsItemBytes = 16;   // LDS ahead of the bodies' LDS in the persistent launch

template <typename T, int N, int NT, typename FX, typename FY, typename FZ>
__global__ __launch_bounds__(NT) void k_persist(const T* in, cplx<T>* __restrict__ W2, T* out, T* removed, PsArgs a,
                                               ZpArgs za,
                                               const cplx<T>* __restrict__ twx, const cplx<T>* __restrict__ twy,
                                               const cplx<T>* __restrict__ twz, const double* __restrict__ symu,
                                               T scale) {
  // the claimed item sits in the first 16 bytes of the dynamic LDS and the bodies' LDS after
  // it: a static __shared__ variable would put the dynamic LDS at its end (byte 4), and every
  // 8-byte LDS access of the bodies would be misaligned
  extern __shared__ unsigned char smem_raw[];
  int& s_item = *reinterpret_cast<int*>(smem_raw);
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw + kPsItemBytes);
  const int fplanes = 6 * a.nz;                       // planes of one field
  const int planes = a.batch * fplanes;
  const int ntile = zproj_tiles(za);
  const int total = a.batch * (2 * a.nP + a.nZ);
  unsigned* ctr = a.ctr;
  // Wave 0 keeps the queue and the counters, with branches on a wave-uniform value only: a
  // branch on the thread index next to a barrier lets the compiler merge the publish of one
  // item with the claim of the next into one thread-0 region that the other lanes skip, and
  // then the other waves pass the barrier at the top of the loop before the claim.  Each
  // counter operation runs on the whole wave and adds lane 0's one (the others add zero).
  const bool w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x) < 64;
  const unsigned one = (threadIdx.x & 63) == 0 ? 1u : 0u;
  for (;;) {
    if (w0) s_item = __builtin_amdgcn_readfirstlane((int)atomicAdd(&ctr[0], one));
    __syncthreads();
    // the item is read into a scalar register, so the loop exit and the stage branches are
    // uniform for the compiler too
    const int q = __builtin_amdgcn_readfirstlane(s_item);
    if (q >= total) break;
    int stage = 0, b = 0, j = 0;
    ps_decode(a, q, stage, b, j);
    // the thread index passes through an empty asm per item, so that no body's index
    // arithmetic is hoisted out of the item loop (it would stay live across the others)
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (stage > 0) {
      if (w0) {
        unsigned* cnt = &ctr[4 + (stage == 1 ? 0 : a.batch) + b];
        const unsigned need = stage == 1 ? (unsigned)a.nP : (unsigned)a.nZ;
        unsigned polls = 0;
        while ((unsigned)__builtin_amdgcn_readfirstlane(
                   (int)__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < need) {
          // give up past the limit, or at once when another wait already has
          if (++polls > a.spin_limit ||
              ((polls & 255u) == 0 &&
               __builtin_amdgcn_readfirstlane(
                   (int)__hip_atomic_load(&ctr[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)) {
            atomicOr(&ctr[2], one);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
    }
    if (stage == 1) {
      for (int k = 0; k < a.gt; ++k) {
        const int tile = j * a.gt + k;
        if (tile < ntile) zproj_body<T, FZ>(W2, za, twz, symu, tile, b, lds, tid);
        __syncthreads();
      }
    } else {
      for (int k = 0; k < a.gp; ++k) {
        const int pf = j * a.gp + k;
        if (pf < fplanes) {
          const int plane = b * fplanes + pf;
          if (stage == 0) plane_r2c_body<T, N, N, NT, FX, FY>(in, W2, plane, planes, twx, twy, lds, tid);
          else plane_c2r_body<T, N, N, NT, FX, FY>(W2, out, in, removed, plane, planes, twx, twy, scale, lds, tid);
        }
        __syncthreads();
      }
    }
    if (stage < 2) {
      // every wave's stores complete before the item is published
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (w0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        atomicAdd(&ctr[4 + (stage == 0 ? 0 : a.batch) + b], one);
      }
    }
  }
  // the last workgroup to finish resets the counters for the next launch: every other one has
  // made its final claim, so nothing reads them any more
  if (w0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned done = (unsigned)__builtin_amdgcn_readfirstlane((int)atomicAdd(&ctr[1], one));
    if (done == gridDim.x - 1) {
      for (int i = (int)(threadIdx.x & 63); i < 2 * a.batch; i += 64)
        __hip_atomic_store(&ctr[4 + i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (one) {
        __hip_atomic_store(&ctr[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctr[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// ------------------------------------------------------------ dispatch -----

// radix-8 stages throughout (radix 16 needs more registers than a resident plane leaves)
template <typename T, int N> struct PlaneCfg;
template <> struct PlaneCfg<float, 64> { static constexpr int NT = 256; using FX = Sched<8, 8>; using FY = FX; };
template <> struct PlaneCfg<float, 128> { static constexpr int NT = 256; using FX = Sched<8, 8, 2>; using FY = FX; };
template <> struct PlaneCfg<float, 256> {
  static constexpr int NT = 1024; using FX = Sched<8, 8, 4>; using FY = Sched<8, 8, 4>;
};
template <> struct PlaneCfg<double, 64> { static constexpr int NT = 256; using FX = Sched<8, 8>; using FY = FX; };
template <> struct PlaneCfg<double, 128> { static constexpr int NT = 512; using FX = Sched<8, 8, 2>; using FY = FX; };
template <> struct PlaneCfg<double, 256> { static constexpr int NT = 512; using FX = Sched<8, 8, 4>; using FY = FX; };

// z schedules: eight elements per thread in FP32, four in FP64 (six components of them
// stay in registers across the projection)
template <typename T, int NZ> struct ZCfg;
template <> struct ZCfg<float, 64> { using F = Sched<8, 8>; };
template <> struct ZCfg<float, 128> { using F = Sched<8, 8, 2>; };
template <> struct ZCfg<float, 256> { using F = Sched<8, 8, 4>; };
template <> struct ZCfg<double, 64> { using F = Sched<4, 4, 4>; };
template <> struct ZCfg<double, 128> { using F = Sched<4, 4, 4, 2>; };
template <> struct ZCfg<double, 256> { using F = Sched<4, 4, 4, 4>; };
// four elements per thread in FP32: half the registers (the persistent launch's z stage)
template <typename T, int NZ> struct ZCfg4;
template <> struct ZCfg4<float, 64> { using F = Sched<4, 4, 4>; };
template <> struct ZCfg4<float, 128> { using F = Sched<4, 4, 4, 2>; };
template <> struct ZCfg4<float, 256> { using F = Sched<4, 4, 4, 4>; };

template <typename T, int N>
size_t plane_lds_bytes() {
  using Cf = PlaneCfg<T, N>;
  return PlaneShape<T, N, N, Cf::NT, typename Cf::FX, typename Cf::FY>::lds_elems * sizeof(cplx<T>);
}

// Workgroups above 64 KB of dynamic LDS need the function attribute raised first.
hipError_t allow_lds(const void* kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T, int N>
hipError_t plane_r2c_n(const T* in, cplx<T>* W2, const Geom& g, const cplx<T>* twx, const cplx<T>* twy,
                       hipStream_t s) {
  using Cf = PlaneCfg<T, N>;
  using FX = typename Cf::FX;
  using FY = typename Cf::FY;
  const size_t lds = plane_lds_bytes<T, N>();
  static const hipError_t once = allow_lds(reinterpret_cast<const void*>(&k_plane_r2c<T, N, N, Cf::NT, FX, FY>), lds);
  if (once != hipSuccess) return once;
  hipLaunchKernelGGL((k_plane_r2c<T, N, N, Cf::NT, FX, FY>), dim3(g.batch * 6 * g.nz), dim3(Cf::NT), lds, s, in, W2,
                     twx, twy);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t plane_c2r_n(const cplx<T>* W2, T* out, const T* in, T* removed, const Geom& g, const cplx<T>* twx,
                       const cplx<T>* twy, hipStream_t s) {
  using Cf = PlaneCfg<T, N>;
  using FX = typename Cf::FX;
  using FY = typename Cf::FY;
  const size_t lds = plane_lds_bytes<T, N>();
  static const hipError_t once = allow_lds(reinterpret_cast<const void*>(&k_plane_c2r<T, N, N, Cf::NT, FX, FY>), lds);
  if (once != hipSuccess) return once;
  const T scale = (T)(1.0 / ((double)g.nx * g.ny * g.nz));
  hipLaunchKernelGGL((k_plane_c2r<T, N, N, Cf::NT, FX, FY>), dim3(g.batch * 6 * g.nz), dim3(Cf::NT), lds, s, W2, out,
                     in, removed, twx, twy, scale);
  return hipGetLastError();
}

template <typename T, int NZ, typename F = typename ZCfg<T, NZ>::F>
hipError_t zproj_n(cplx<T>* W2, const Geom& g, const cplx<T>* twz, const double* symu, int tc, hipStream_t s) {
  const ZpArgs a{g.nx, g.ny, g.nz, tc, g.batch};
  if ((double)6 * NZ * g.ny * (g.nx / 2) * sizeof(cplx<T>) >= 4294967296.0) return hipErrorInvalidValue;  // 32-bit offsets
  if (tc < 1 || g.ny % tc != 0 || tc * (NZ / F::E) > kMaxFastThreads) return hipErrorInvalidValue;
  const size_t lds = 2 * (size_t)tc * (NZ + (NZ >> kSkew) + 1) * sizeof(cplx<T>);
  static const hipError_t once = allow_lds(reinterpret_cast<const void*>(&k_zproj<T, F>), 160 * 1024);
  if (once != hipSuccess && lds > 64 * 1024) return once;
  const int ntile = g.ny * (g.nx / 2) / tc + g.ny / tc;
  hipLaunchKernelGGL((k_zproj<T, F>), dim3(ntile * g.batch), dim3(tc * (NZ / F::E)), lds, s, W2, a, twz, symu);
  return hipGetLastError();
}

bool plane_edge_ok(int n) { return n == 64 || n == 128 || n == 256; }

// Persistent launch: one workgroup shape for all three stages (the plane kernel's), so the z
// tiles are NT / (NZ / E) columns wide.
// Plane shape of the persistent launch: 512 threads at 128 (half the plane registers per thread
// of the 256-thread pass kernel; the transforms, and so the results, are the same).
template <typename T, int N> struct PersistPlaneCfg : PlaneCfg<T, N> {};
template <> struct PersistPlaneCfg<float, 128> { static constexpr int NT = 512; using FX = Sched<8, 8, 2>; using FY = FX; };

template <typename T, int N, int NZ>
hipError_t persist_n(const T* in, cplx<T>* W2, T* out, T* removed, const Geom& g, const cplx<T>* twx,
                     const cplx<T>* twy, const cplx<T>* twz, const double* symu, unsigned* ctr, hipStream_t s) {
  using Cf = PersistPlaneCfg<T, N>;
  using FX = typename Cf::FX;
  using FY = typename Cf::FY;
  using FZ = typename ZCfg4<T, NZ>::F;
  constexpr int NT = Cf::NT, PZ = NZ / FZ::E, TC = NT / PZ;
  static_assert(TC >= 1 && N % TC == 0, "z tiles must divide the Nyquist column count");
  if ((double)6 * NZ * g.ny * (g.nx / 2) * sizeof(cplx<T>) >= 4294967296.0) return hipErrorInvalidValue;  // 32-bit offsets
  const ZpArgs za{g.nx, g.ny, g.nz, TC, g.batch};
  PsArgs a{};
  a.batch = g.batch;
  a.nz = g.nz;
  // items of about 64 K elements (a plane item) or one z tile; four times that from eight
  // fields on, where the batch fills the device anyway and each item's claim, publish and
  // L2 writeback and invalidate are paid a quarter as often
  const int m = g.batch >= 8 ? 4 : 1;
  a.gp = m * (N * N >= 16384 ? 1 : 16384 / (N * N));
  a.gt = m;
  a.nP = (6 * g.nz + a.gp - 1) / a.gp;
  a.nZ = (zproj_tiles(za) + a.gt - 1) / a.gt;
  a.ctr = ctr;
  // polls before a wait gives up; EQ_PERSIST_SPIN_LIMIT lowers it so that tests can force the
  // reported failure while every wait still ends
  a.spin_limit = 1u << 18;
  if (const char* e = std::getenv("EQ_PERSIST_SPIN_LIMIT")) {
    const long v = std::atol(e);
    if (v >= 1 && v < (long)a.spin_limit) a.spin_limit = (unsigned)v;
  }
  const size_t lds = kPsItemBytes + std::max(PlaneShape<T, N, N, NT, FX, FY>::lds_elems * sizeof(cplx<T>),
                                             zproj_lds(g, sizeof(T) == 8, TC));
  const void* k = reinterpret_cast<const void*>(&k_persist<T, N, NT, FX, FY, FZ>);
  static const hipError_t once = allow_lds(k, lds);
  if (once != hipSuccess) return once;
  // as many workgroups as the device holds at once, at most one per item
  static const int cap = [&] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, NT, lds) != hipSuccess)
      return 256;
    return std::max(1, cus * per);
  }();
  const int total = g.batch * (2 * a.nP + a.nZ);
  const int grid = std::max(1, std::min(cap, total));
  // lag: one step, plus as many as the grid's items in flight cover
  const int step_items = 2 * a.nP + a.nZ;
  a.lag = 1 + (grid + step_items - 1) / step_items;
  const T scale = (T)(1.0 / ((double)g.nx * g.ny * g.nz));
  hipLaunchKernelGGL((k_persist<T, N, NT, FX, FY, FZ>), dim3(grid), dim3(NT), lds, s, in, W2, out, removed, a, za, twx,
                     twy, twz, symu, scale);
  return hipGetLastError();
}

}  // namespace

bool persist_route_supported(const Geom& g, bool fp64) {
  return !fp64 && g.nx == g.ny && (g.nx == 64 || g.nx == 128) && plane_edge_ok(g.nz);
}

template <typename T>
hipError_t launch_persist(const T* in, cplx<T>* W2, T* out, T* removed, const Geom& g, const cplx<T>* twx,
                          const cplx<T>* twy, const cplx<T>* twz, const double* symu, unsigned* ctr, hipStream_t s) {
  static_assert(sizeof(T) == 4, "the persistent launch is FP32");
  if (!persist_route_supported(g, false)) return hipErrorInvalidValue;
  if (g.nx == 64) {
    switch (g.nz) {
      case 64: return persist_n<T, 64, 64>(in, W2, out, removed, g, twx, twy, twz, symu, ctr, s);
      case 128: return persist_n<T, 64, 128>(in, W2, out, removed, g, twx, twy, twz, symu, ctr, s);
      default: return persist_n<T, 64, 256>(in, W2, out, removed, g, twx, twy, twz, symu, ctr, s);
    }
  }
  switch (g.nz) {
    case 64: return persist_n<T, 128, 64>(in, W2, out, removed, g, twx, twy, twz, symu, ctr, s);
    case 128: return persist_n<T, 128, 128>(in, W2, out, removed, g, twx, twy, twz, symu, ctr, s);
    default: return persist_n<T, 128, 256>(in, W2, out, removed, g, twx, twy, twz, symu, ctr, s);
  }
}

bool plane_route_supported(const Geom& g, bool fp64) {
  if (g.nx != g.ny || !plane_edge_ok(g.nx) || !plane_edge_ok(g.nz)) return false;
  return !fp64 || g.nx <= 128;      // an FP64 256^2 plane (528 KB) does not fit one CU
}

size_t plane_lds(const Geom& g, bool fp64) {
  switch (g.nx) {
    case 64: return fp64 ? plane_lds_bytes<double, 64>() : plane_lds_bytes<float, 64>();
    case 128: return fp64 ? plane_lds_bytes<double, 128>() : plane_lds_bytes<float, 128>();
    default: return fp64 ? plane_lds_bytes<double, 256>() : plane_lds_bytes<float, 256>();
  }
}

int pick_tc_zproj(const Geom& g, bool fp64, int want, bool e4) {
  const int plane = g.ny;      // tiles must divide the Nyquist columns too (and so every row of W2)
  const int P = g.nz / (fp64 || e4 ? 4 : 8);
  int tc = want > 0 ? want : (fp64 ? 8 : 16);     // 128-byte row segments per component
  if (tc < 1) tc = 1;
  while (tc > 1 && (plane % tc != 0 || tc * P > kMaxFastThreads)) tc >>= 1;
  return tc;
}

size_t zproj_lds(const Geom& g, bool fp64, int tc) {
  return 2 * (size_t)tc * (g.nz + (g.nz >> kSkew) + 1) * (fp64 ? 16 : 8);
}

template <typename T>
hipError_t launch_plane_r2c(const T* in, cplx<T>* W2, const Geom& g, const cplx<T>* twx, const cplx<T>* twy,
                            hipStream_t s) {
  switch (g.nx) {
    case 64: return plane_r2c_n<T, 64>(in, W2, g, twx, twy, s);
    case 128: return plane_r2c_n<T, 128>(in, W2, g, twx, twy, s);
    case 256:
      if constexpr (sizeof(T) == 4) return plane_r2c_n<T, 256>(in, W2, g, twx, twy, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_plane_c2r(const cplx<T>* W2, T* out, const T* in, T* removed, const Geom& g, const cplx<T>* twx,
                            const cplx<T>* twy, hipStream_t s) {
  switch (g.nx) {
    case 64: return plane_c2r_n<T, 64>(W2, out, in, removed, g, twx, twy, s);
    case 128: return plane_c2r_n<T, 128>(W2, out, in, removed, g, twx, twy, s);
    case 256:
      if constexpr (sizeof(T) == 4) return plane_c2r_n<T, 256>(W2, out, in, removed, g, twx, twy, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_zproj(cplx<T>* W2, const Geom& g, const cplx<T>* twz, const double* symu, int tc, bool e4,
                        hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (e4) {
      switch (g.nz) {
        case 64: return zproj_n<T, 64, typename ZCfg4<T, 64>::F>(W2, g, twz, symu, tc, s);
        case 128: return zproj_n<T, 128, typename ZCfg4<T, 128>::F>(W2, g, twz, symu, tc, s);
        case 256: return zproj_n<T, 256, typename ZCfg4<T, 256>::F>(W2, g, twz, symu, tc, s);
        default: return hipErrorInvalidValue;
      }
    }
  }
  switch (g.nz) {
    case 64: return zproj_n<T, 64>(W2, g, twz, symu, tc, s);
    case 128: return zproj_n<T, 128>(W2, g, twz, symu, tc, s);
    case 256: return zproj_n<T, 256>(W2, g, twz, symu, tc, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_plane_r2c<float>(const float*, cplx<float>*, const Geom&, const cplx<float>*,
                                            const cplx<float>*, hipStream_t);
template hipError_t launch_plane_r2c<double>(const double*, cplx<double>*, const Geom&, const cplx<double>*,
                                             const cplx<double>*, hipStream_t);
template hipError_t launch_plane_c2r<float>(const cplx<float>*, float*, const float*, float*, const Geom&,
                                            const cplx<float>*, const cplx<float>*, hipStream_t);
template hipError_t launch_plane_c2r<double>(const cplx<double>*, double*, const double*, double*, const Geom&,
                                             const cplx<double>*, const cplx<double>*, hipStream_t);
template hipError_t launch_zproj<float>(cplx<float>*, const Geom&, const cplx<float>*, const double*, int, bool,
                                        hipStream_t);
template hipError_t launch_persist<float>(const float*, cplx<float>*, float*, float*, const Geom&, const cplx<float>*,
                                          const cplx<float>*, const cplx<float>*, const double*, unsigned*, hipStream_t);

template hipError_t launch_zproj<double>(cplx<double>*, const Geom&, const cplx<double>*, const double*, int, bool,
                                         hipStream_t);

}  // namespace eq
