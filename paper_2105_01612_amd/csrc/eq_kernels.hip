// eq_kernels.hip -- gfx950 kernels of the equilibrium projection and their launchers.
//
// Pass schedule of one projection (Section 3.3 solution strategy, evaluated in
// Fourier space as in Section 4):
//   z_r2c  real field -> Hermitian half spectrum along z (two real x-columns are
//          packed into one complex line and separated after the transform)
//   y fwd  complex DFT along y
//   x proj complex DFT along x, per-frequency projection P A P over all six
//          components of the frequency, inverse DFT along x (one read, one write)
//   y inv  inverse DFT along y
//   z_c2r  Hermitian half -> real along z, 1/(nx ny nz), optional removed part
// Each pass reads its tile once and writes it once.  Strided passes (y, z) tile
// over contiguous x with lanes running along x, so every global access is a
// contiguous run of tile-width elements; the x pass reads whole rows.
//
// Register-engine kernels (eq_kernels_impl.hpp) issue all E global loads of a
// thread's line segment back to back, run the first FFT stage on them in
// registers, exchange through LDS between stages, and store the last stage's
// registers directly; their radix schedule is compile-time for the common edges
// (eq_sched_*.hip) and read at run time otherwise.  Generic kernels (suffix _g,
// this file) stage whole tiles through LDS; they serve edges the register engine
// does not schedule.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <mutex>

#include "eq_fft.hpp"
#include "eq_internal.hpp"
#include "eq_kernels_impl.hpp"

namespace eq {

namespace {

// ------------------------------------------------------------- tables ------

__global__ void k_tables(int nx, int ny, int nz, int op, double h, double* __restrict__ sym,
                         double2* __restrict__ tw64, float2* __restrict__ tw32) {
  const int total = nx + ny + nz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    int n, q;
    if (i < nx) { n = nx; q = i; }
    else if (i < nx + ny) { n = ny; q = i - nx; }
    else { n = nz; q = i - nx - ny; }
    // twiddle exp(-2 pi i q / n), FP64 on the device (sincospi is exact at multiples of 1/2)
    double sn, cs;
    sincospi(2.0 * (double)q / (double)n, &sn, &cs);
    tw64[i] = make_double2(cs, -sn);
    tw32[i] = make_float2((float)cs, (float)(-sn));
    // derivative symbol of the operator (Section 4.1 eq:cdo, Section 4.2 eq:diff); sym[total + i]
    // holds the same symbol for h = 1, which the projection uses (it depends on the direction only)
    double su;
    if (op == 0) {
      const int k = (2 * q < n) ? q : ((2 * q == n) ? 0 : q - n);
      su = 2.0 * M_PI * (double)k / (double)n;
    } else {
      su = ((2 * q) % n == 0) ? 0.0 : sinpi(2.0 * (double)q / (double)n);
    }
    sym[i] = su / h;
    sym[total + i] = su;
  }
}

// ------------------------------------------------------- generic kernels ---

template <typename T, int E>
__global__ __launch_bounds__(kMaxThreads) void k_z_r2c_g(const T* __restrict__ in, cplx<T>* __restrict__ W, ZArgs a,
                                                         FftDesc d, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int ntx = a.nx / a.tx;
  int bid = blockIdx.x;
  const int xt = bid % ntx; bid /= ntx;
  const int y = bid % a.ny;
  const int bc = bid / a.ny;
  const int np = a.tx >> 1;
  const int nz = a.nz, nzh = nz / 2 + 1;
  const size_t plane = (size_t)a.ny * a.nx;
  const T* src = in + (size_t)bc * nz * plane + (size_t)y * a.nx + (size_t)xt * a.tx;
  for (int u = threadIdx.x; u < nz * np; u += blockDim.x) {
    const int z = u / np, j = u - z * np;
    if (!a.e.on) {
      lds[u] = *reinterpret_cast<const C*>(src + (size_t)z * plane + 2 * j);
    } else {
      const EmbedPair ep = embed_pair(a.e, y, xt * a.tx + 2 * j);
      const T* s = in + (size_t)bc * nz * ep.plane + (size_t)z * ep.plane;
      lds[u] = mk<T>(ep.ok0 ? s[ep.off0] : (T)0, ep.ok1 ? s[ep.off1] : (T)0);
    }
  }
  __syncthreads();
  fft_lines<T, E, false>(lds, np, 1, np, d, tw, threadIdx.x);
  C* dst = W + (size_t)bc * nzh * plane + (size_t)y * a.nx + (size_t)xt * a.tx;
  const T half = (T)0.5;
  for (int u = threadIdx.x; u < nzh * np; u += blockDim.x) {
    const int kz = u / np, j = u - kz * np;
    const C Z = lds[kz * np + j];
    const C Zm = lds[((nz - kz) % nz) * np + j];
    C* o = dst + (size_t)kz * plane + 2 * j;
    o[0] = mk<T>((Z.x + Zm.x) * half, (Z.y - Zm.y) * half);
    o[1] = mk<T>((Z.y + Zm.y) * half, (Zm.x - Z.x) * half);
  }
}

template <typename T, int E>
__global__ __launch_bounds__(kMaxThreads) void k_z_c2r_g(const cplx<T>* __restrict__ W, T* out, const T* in,
                                                         T* removed, ZcArgs a, FftDesc d,
                                                         const cplx<T>* __restrict__ tw, T scale) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int ntx = a.nx / a.tx;
  int bid = blockIdx.x;
  const int xt = bid % ntx; bid /= ntx;
  const int y = bid % a.ny; bid /= a.ny;
  const int c = bid % a.ncomp;
  const int b = bid / a.ncomp;
  const int np = a.tx >> 1;
  const int nz = a.nz, nzh = nz / 2 + 1, nyq = nz / 2;
  const size_t plane = (size_t)a.ny * a.nx;
  const C* src = W + ((size_t)(b * 6 + c) * nzh) * plane + (size_t)y * a.nx + (size_t)xt * a.tx;
  for (int u = threadIdx.x; u < nzh * np; u += blockDim.x) {
    const int kz = u / np, j = u - kz * np;
    const C* s = src + (size_t)kz * plane + 2 * j;
    C A = s[0], B = s[1];
    if (kz == 0 || kz == nyq) { A.y = (T)0; B.y = (T)0; }
    lds[kz * np + j] = mk<T>(A.x - B.y, A.y + B.x);
    if (kz > 0 && kz < nyq) lds[(nz - kz) * np + j] = mk<T>(A.x + B.y, B.x - A.y);
  }
  __syncthreads();
  fft_lines<T, E, true>(lds, np, 1, np, d, tw, threadIdx.x);
  const size_t obase = (size_t)b * a.out_field + (size_t)c * a.out_comp + (size_t)y * a.nx + (size_t)xt * a.tx;
  for (int u = threadIdx.x; u < nz * np; u += blockDim.x) {
    const int z = u / np, j = u - z * np;
    const C Z = lds[u];
    if (a.e.on) {
      const EmbedPair ep = embed_pair(a.e, y, xt * a.tx + 2 * j);
      const size_t o = (size_t)b * a.out_field + (size_t)c * a.out_comp + (size_t)z * ep.plane;
      const T o0 = Z.x * scale, o1 = Z.y * scale;
      if (ep.ok0) {
        if (removed) removed[o + ep.off0] = in[o + ep.off0] - o0;
        out[o + ep.off0] = o0;
      }
      if (ep.ok1) {
        if (removed) removed[o + ep.off1] = in[o + ep.off1] - o1;
        out[o + ep.off1] = o1;
      }
      continue;
    }
    const size_t off = obase + (size_t)z * plane + 2 * j;
    C o = mk<T>(Z.x * scale, Z.y * scale);
    if (removed) {
      const C s = *reinterpret_cast<const C*>(in + off);
      *reinterpret_cast<C*>(removed + off) = mk<T>(s.x - o.x, s.y - o.y);
    }
    *reinterpret_cast<C*>(out + off) = o;
  }
}

template <typename T, int E, bool INV>
__global__ __launch_bounds__(kMaxThreads) void k_y_g(cplx<T>* __restrict__ W, YArgs a, FftDesc d,
                                                     const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C* base = W + y_tile_base(a);
  const int tx = a.tx;
  for (int u = threadIdx.x; u < a.ny * tx; u += blockDim.x) {
    const int y = u / tx, x = u - y * tx;
    lds[u] = base[(size_t)y * a.nx + x];
  }
  __syncthreads();
  fft_lines<T, E, INV>(lds, tx, 1, tx, d, tw, threadIdx.x);
  for (int u = threadIdx.x; u < a.ny * tx; u += blockDim.x) {
    const int y = u / tx, x = u - y * tx;
    base[(size_t)y * a.nx + x] = lds[u];
  }
}

template <typename T, int E>
__global__ __launch_bounds__(kMaxThreads) void k_x_g(cplx<T>* __restrict__ W, XArgs a, FftDesc d,
                                                     const cplx<T>* __restrict__ tw, const double* __restrict__ sym) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int nx = a.nx, ls = nx + 1, rw = a.rw;
  const int row0 = blockIdx.x * rw;
  const int nrows = min(rw, a.rows - row0);
  const int ncomp_out = (a.mode & (XM_DIV | XM_DISP)) ? 3 : 6;
  int kz, ky;
  for (int c = 0; c < 6; ++c) {
    for (int u = threadIdx.x; u < rw * nx; u += blockDim.x) {
      const int r = u / nx, x = u - r * nx;
      C v = mk<T>((T)0, (T)0);
      if (r < nrows) v = W[x_row_base(a, row0 + r, c, kz, ky) + x];
      lds[(c * rw + r) * ls + x] = v;
    }
  }
  __syncthreads();
  if (a.mode & XM_FWD) fft_lines<T, E, false>(lds, 6 * rw, ls, 1, d, tw, threadIdx.x);
  if (a.mode & (XM_PROJ | XM_DIV | XM_DISP)) {
    const double* symx = sym;
    const double* symy = sym + nx;
    const double* symz = sym + nx + a.ny;
    for (int u = threadIdx.x; u < nrows * nx; u += blockDim.x) {
      const int r = u / nx, kx = u - r * nx;
      (void)x_row_base(a, row0 + r, 0, kz, ky);
      C A[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) A[c] = lds[(c * rw + r) * ls + kx];
      if (a.mode & XM_PROJ) {
        project_one<T>(A, symx[kx], symy[ky], symz[kz]);
#pragma unroll
        for (int c = 0; c < 6; ++c) lds[(c * rw + r) * ls + kx] = A[c];
      } else {
        vector_op<T>(a.mode, A, symx[kx], symy[ky], symz[kz], a.h);
#pragma unroll
        for (int c = 0; c < 3; ++c) lds[(c * rw + r) * ls + kx] = A[c];
      }
    }
    __syncthreads();
  }
  if (a.mode & XM_INV) fft_lines<T, E, true>(lds, ncomp_out * rw, ls, 1, d, tw, threadIdx.x);
  for (int c = 0; c < ncomp_out; ++c) {
    for (int u = threadIdx.x; u < nrows * nx; u += blockDim.x) {
      const int r = u / nx, x = u - r * nx;
      W[x_row_base(a, row0 + r, c, kz, ky) + x] = lds[(c * rw + r) * ls + x];
    }
  }
}

// ------------------------------------------------------------ residual -----

constexpr int kRedThreads = 256;

// A value every lane holds alike, moved to scalar registers (exact: lane 0's copy).
__device__ __forceinline__ double uniform_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Deterministic block reduction of the kRedWidth record (sums, except [1] = max).
__device__ __forceinline__ void block_reduce_record(double* v, double* sh /* kRedWidth * kRedThreads */) {
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kRedWidth; ++k) sh[k * kRedThreads + t] = v[k];
  __syncthreads();
  for (int stride = kRedThreads / 2; stride > 0; stride >>= 1) {
    if (t < stride) {
#pragma unroll
      for (int k = 0; k < kRedWidth; ++k) {
        const double o = sh[k * kRedThreads + t + stride];
        double& mm = sh[k * kRedThreads + t];
        mm = (k == 1) ? fmax(mm, o) : mm + o;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kRedWidth; ++k) v[k] = sh[k * kRedThreads];
}

struct DArgs {
  int nx, ny, nz;
  int tx, ty;            // tx * ty threads (== kRedThreads) cover a tx by 2 * ty tile
  int tiles_x, tiles;    // tiles per plane
  int zc;                // z chunks: a work item is (tile, z chunk)
  double inv2h;
};

template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T x, y;
};

// Element e of component c of one field: a raw buffer load when every component's byte
// range fits the 32-bit offset (the six resources sit in SGPRs and one 32-bit offset per
// neighbour serves all six components), else a plain load.
template <typename T, bool BUF>
struct FieldReader {
  const T* f[6];
  __amdgpu_buffer_rsrc_t r[6];
  __device__ FieldReader(const T* F, size_t M) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      f[c] = F + c * M;
      if constexpr (BUF) r[c] = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(f[c]), 0, (int)(M * sizeof(T)), kBufWord3);
    }
  }
  // elements e and e + 1 (e even: 8-byte aligned in FP32, 16-byte in FP64), unconverted
  __device__ __forceinline__ Pair<T> raw2(int c, size_t e) const {
    Pair<T> v;
    if constexpr (BUF) {
      const unsigned off = (unsigned)e * (unsigned)sizeof(T);
      if constexpr (sizeof(T) == 4) {
        const auto r2 = __builtin_amdgcn_raw_buffer_load_b64(r[c], off, 0, 0);
        __builtin_memcpy(&v, &r2, sizeof(v));
      } else {
        const auto r2 = __builtin_amdgcn_raw_buffer_load_b128(r[c], off, 0, 0);
        __builtin_memcpy(&v, &r2, sizeof(v));
      }
    } else {
      v = *reinterpret_cast<const Pair<T>*>(f[c] + e);
    }
    return v;
  }
  // the stored value, unconverted
  __device__ __forceinline__ T raw(int c, size_t e) const {
    if constexpr (BUF) {
      const unsigned off = (unsigned)e * (unsigned)sizeof(T);
      if constexpr (sizeof(T) == 4) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r[c], off, 0, 0));
      } else {
        const auto raw = __builtin_amdgcn_raw_buffer_load_b64(r[c], off, 0, 0);
        double v;
        __builtin_memcpy(&v, &raw, sizeof(v));
        return v;
      }
    } else {
      return f[c][e];
    }
  }
  __device__ __forceinline__ double operator()(int c, size_t e) const {
    if constexpr (BUF) {
      const unsigned off = (unsigned)e * (unsigned)sizeof(T);
      if constexpr (sizeof(T) == 4) {
        return (double)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r[c], off, 0, 0));
      } else {
        const auto raw = __builtin_amdgcn_raw_buffer_load_b64(r[c], off, 0, 0);
        double v;
        __builtin_memcpy(&v, &raw, sizeof(v));
        return v;
      }
    } else {
      return (double)f[c][e];
    }
  }
};

// DDO divergence in real space: periodic central differences, exactly the DDO symbol.
// A thread owns rows y and y + 1 of one x column of a z chunk and marches along z: the
// three components differentiated along z (S33, S23, S13) roll through registers, each
// row is the other's y neighbour for S12, S22 and S23, and only rows y - 1 and y + 2
// come from neighbouring tiles (15 loads per voxel instead of 18).
template <typename T, bool BUF>
__global__ __launch_bounds__(kRedThreads) void k_div_ddo(const T* __restrict__ S, T* __restrict__ div,
                                                         double* __restrict__ partials, DArgs a) {
  __shared__ double sh[kRedWidth * kRedThreads];
  const int b = blockIdx.y;
  const size_t M = (size_t)a.nx * a.ny * a.nz;
  const size_t sz = (size_t)a.nx * a.ny;
  const FieldReader<T, BUF> F(S + (size_t)b * 6 * M, M);
  double acc[kRedWidth];
#pragma unroll
  for (int k = 0; k < kRedWidth; ++k) acc[k] = 0.0;
  // the component sums are taken about the field's first voxel, so the variance of a field
  // whose mean is large against its spread does not cancel (sum d^2 - (sum d)^2 / M, d = S - shift);
  // the shifts are the same in every lane and are kept in scalar registers
  const double sh0 = uniform_f64(F(0, 0)), sh1 = uniform_f64(F(1, 0)), sh2 = uniform_f64(F(2, 0));
  const double sh3 = uniform_f64(F(3, 0)), sh4 = uniform_f64(F(4, 0)), sh5 = uniform_f64(F(5, 0));
  const int lx = threadIdx.x % a.tx, ly = threadIdx.x / a.tx;
  const int items = a.tiles * a.zc;
  // each XCD takes a contiguous run of work items, so the y-halo rows of neighbouring
  // tiles are read from its own L2
  const int lb = xcd_contiguous(blockIdx.x, gridDim.x);
  for (int it = lb; it < items; it += gridDim.x) {
    const int tile = it % a.tiles, zi = it / a.tiles;
    const int x = (tile % a.tiles_x) * a.tx + lx;
    const int y = (tile / a.tiles_x) * (2 * a.ty) + 2 * ly;       // even; ny is even, so y + 1 < ny
    const int z0 = (int)(((long)zi * a.nz) / a.zc), z1 = (int)(((long)(zi + 1) * a.nz) / a.zc);
    if (x >= a.nx || y >= a.ny || z0 >= z1) continue;
    // in-plane offsets, fixed along the march: rows a = y, b = y + 1; outer rows y - 1, y + 2
    const size_t ca = (size_t)y * a.nx + x, cb = ca + a.nx;
    const size_t ym = (y == 0) ? ca + sz - a.nx : ca - a.nx;
    const size_t yq = (y + 2 == a.ny) ? ca + 2 * a.nx - sz : ca + 2 * a.nx;
    const long dxp = (x + 1 == a.nx) ? 1 - (long)a.nx : 1;
    const long dxm = (x == 0) ? (long)a.nx - 1 : -1;
    const size_t pm = (size_t)(z0 == 0 ? a.nz - 1 : z0 - 1) * sz;
    const size_t p0 = (size_t)z0 * sz;
    double a2m = F(2, pm + ca), a3m = F(3, pm + ca), a4m = F(4, pm + ca);
    double a2c = F(2, p0 + ca), a3c = F(3, p0 + ca), a4c = F(4, p0 + ca);
    double b2m = F(2, pm + cb), b3m = F(3, pm + cb), b4m = F(4, pm + cb);
    double b2c = F(2, p0 + cb), b3c = F(3, p0 + cb), b4c = F(4, p0 + cb);
    // the 30 values one plane step reads (rows a = y, b = y + 1): centres of S11, S22, S12;
    // x neighbours of S11, S12, S13; the outer y rows of S12, S22, S23; the next plane of S33,
    // S23, S13.  FP32 fields load the step after next while the current one is evaluated.
    auto load_step = [&](int z, T* v) {
      const size_t p = (size_t)z * sz;
      const size_t pn = (size_t)(z + 1 == a.nz ? 0 : z + 1) * sz;
      const size_t qa = p + ca, qb = p + cb;
      v[0] = F.raw(0, qa); v[1] = F.raw(1, qa); v[2] = F.raw(5, qa);
      v[3] = F.raw(0, qb); v[4] = F.raw(1, qb); v[5] = F.raw(5, qb);
      v[6] = F.raw(0, qa + dxp); v[7] = F.raw(0, qa + dxm); v[8] = F.raw(5, qa + dxp); v[9] = F.raw(5, qa + dxm);
      v[10] = F.raw(4, qa + dxp); v[11] = F.raw(4, qa + dxm);
      v[12] = F.raw(0, qb + dxp); v[13] = F.raw(0, qb + dxm); v[14] = F.raw(5, qb + dxp); v[15] = F.raw(5, qb + dxm);
      v[16] = F.raw(4, qb + dxp); v[17] = F.raw(4, qb + dxm);
      v[18] = F.raw(5, p + ym); v[19] = F.raw(1, p + ym); v[20] = F.raw(3, p + ym);
      v[21] = F.raw(5, p + yq); v[22] = F.raw(1, p + yq); v[23] = F.raw(3, p + yq);
      v[24] = F.raw(2, pn + ca); v[25] = F.raw(3, pn + ca); v[26] = F.raw(4, pn + ca);
      v[27] = F.raw(2, pn + cb); v[28] = F.raw(3, pn + cb); v[29] = F.raw(4, pn + cb);
    };
    constexpr bool kAhead = sizeof(T) == 4;     // FP64 values would take twice the registers
    T cur[30], nxt[30];
    load_step(z0, cur);
    for (int z = z0; z < z1; ++z) {
      const size_t p = (size_t)z * sz;
      if (kAhead) {
        if (z + 1 < z1) load_step(z + 1, nxt);
      } else if (z > z0) {
        load_step(z, cur);
      }
      const double a0 = cur[0], a1 = cur[1], a5 = cur[2], b0 = cur[3], b1 = cur[4], b5 = cur[5];
      const double a2p = cur[24], a3p = cur[25], a4p = cur[26], b2p = cur[27], b3p = cur[28], b4p = cur[29];
      const size_t qa = p + ca;
      // r_x = d_x S11 + d_y S12 + d_z S13, etc. (slots 0=11 1=22 2=33 3=23 4=13 5=12)
      const double ra0 = (((double)cur[6] - (double)cur[7]) + (b5 - (double)cur[18]) + (a4p - a4m)) * a.inv2h;
      const double ra1 = (((double)cur[8] - (double)cur[9]) + (b1 - (double)cur[19]) + (a3p - a3m)) * a.inv2h;
      const double ra2 = (((double)cur[10] - (double)cur[11]) + (b3c - (double)cur[20]) + (a2p - a2m)) * a.inv2h;
      const double rb0 = (((double)cur[12] - (double)cur[13]) + ((double)cur[21] - a5) + (b4p - b4m)) * a.inv2h;
      const double rb1 = (((double)cur[14] - (double)cur[15]) + ((double)cur[22] - a1) + (b3p - b3m)) * a.inv2h;
      const double rb2 = (((double)cur[16] - (double)cur[17]) + ((double)cur[23] - a3c) + (b2p - b2m)) * a.inv2h;
      const double ma = ra0 * ra0 + ra1 * ra1 + ra2 * ra2;
      const double mb = rb0 * rb0 + rb1 * rb1 + rb2 * rb2;
      acc[0] += ma + mb;
      acc[1] = fmax(acc[1], fmax(ma, mb));
      {
        const double d0 = a0 - sh0, e0 = b0 - sh0, d1 = a1 - sh1, e1 = b1 - sh1;
        const double d2 = a2c - sh2, e2 = b2c - sh2, d3 = a3c - sh3, e3 = b3c - sh3;
        const double d4 = a4c - sh4, e4 = b4c - sh4, d5 = a5 - sh5, e5 = b5 - sh5;
        acc[2] += d0 + e0; acc[8] += d0 * d0 + e0 * e0;
        acc[3] += d1 + e1; acc[9] += d1 * d1 + e1 * e1;
        acc[4] += d2 + e2; acc[10] += d2 * d2 + e2 * e2;
        acc[5] += d3 + e3; acc[11] += d3 * d3 + e3 * e3;
        acc[6] += d4 + e4; acc[12] += d4 * d4 + e4 * e4;
        acc[7] += d5 + e5; acc[13] += d5 * d5 + e5 * e5;
      }
      if (div) {
        T* o = div + (size_t)b * 3 * M + qa;
        o[0] = (T)ra0; o[M] = (T)ra1; o[2 * M] = (T)ra2;
        o[a.nx] = (T)rb0; o[M + a.nx] = (T)rb1; o[2 * M + a.nx] = (T)rb2;
      }
      if (kAhead) {
#pragma unroll
        for (int k = 0; k < 30; ++k) cur[k] = nxt[k];
      }
      a2m = a2c; a3m = a3c; a4m = a4c;
      a2c = a2p; a3c = a3p; a4c = a4p;
      b2m = b2c; b3m = b3c; b4m = b4c;
      b2c = b2p; b3c = b3p; b4c = b4p;
    }
  }
  block_reduce_record(acc, sh);
  if (threadIdx.x == 0) {
    double* pp = partials + ((size_t)b * gridDim.x + blockIdx.x) * kRedWidth;
#pragma unroll
    for (int k = 0; k < kRedWidth; ++k) pp[k] = acc[k];
  }
}

// The same divergence and record for FP64 fields with nx a multiple of 128, with two x
// columns per lane: a wavefront spans 128 columns of rows y and y + 1, each load brings two
// values (16 bytes per lane, half the instructions), and the x neighbours of a lane's pair
// are the next lanes' values (a lane shuffle; lanes 0 and 63 load them when the wavefront
// does not span the whole row).  The four wavefronts of a workgroup take four consecutive
// row pairs, so the outer rows y - 1 and y + 2 of all but two of them are rows the workgroup
// reads itself.  Per-voxel values are those of k_div_ddo bit for bit.  (In FP32 the
// one-column kernel is faster: it holds 12 wavefronts per CU against this kernel's 8.)
struct DvArgs {
  int nx, ny, nz;
  int tiles_x;           // nx / 128
  int tiles;             // tiles_x x groups of 8 rows
  int zc;                // z chunks: a work item is (tile, z chunk)
  double inv2h;
};

template <typename T>
__device__ __forceinline__ T lane_from(T v, int src) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
  } else {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)b);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  }
}

template <typename T, bool BUF>
__global__ __launch_bounds__(kRedThreads) void k_div_ddo2(const T* __restrict__ S, T* __restrict__ div,
                                                          double* __restrict__ partials, DvArgs a) {
  __shared__ double sh[kRedWidth * kRedThreads];
  using P2 = Pair<T>;
  const int b = blockIdx.y;
  const size_t M = (size_t)a.nx * a.ny * a.nz;
  const size_t sz = (size_t)a.nx * a.ny;
  const FieldReader<T, BUF> F(S + (size_t)b * 6 * M, M);
  double acc[kRedWidth];
#pragma unroll
  for (int k = 0; k < kRedWidth; ++k) acc[k] = 0.0;
  // component sums about the field's first voxel, as in k_div_ddo
  const double sh0 = uniform_f64(F(0, 0)), sh1 = uniform_f64(F(1, 0)), sh2 = uniform_f64(F(2, 0));
  const double sh3 = uniform_f64(F(3, 0)), sh4 = uniform_f64(F(4, 0)), sh5 = uniform_f64(F(5, 0));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int src_l = (lane + 63) & 63, src_r = (lane + 1) & 63;
  // lanes 0 and 63 take their outer neighbour from memory unless the wavefront spans the row
  const bool edge_l = a.tiles_x > 1 && lane == 0, edge_r = a.tiles_x > 1 && lane == 63;
  const int items = a.tiles * a.zc;
  const int lb = xcd_contiguous(blockIdx.x, gridDim.x);
  for (int it = lb; it < items; it += gridDim.x) {
    const int tile = it % a.tiles, zi = it / a.tiles;
    const int x0 = (tile % a.tiles_x) * 128 + 2 * lane;
    const int y = (tile / a.tiles_x) * 8 + 2 * w;                   // even; ny is even
    const int z0 = (int)(((long)zi * a.nz) / a.zc), z1 = (int)(((long)(zi + 1) * a.nz) / a.zc);
    if (y >= a.ny || z0 >= z1) continue;                            // uniform in the wavefront
    const size_t ca = (size_t)y * a.nx + x0, cb = ca + a.nx;
    const size_t ym = (y == 0) ? ca + sz - a.nx : ca - a.nx;
    const size_t yq = (y + 2 == a.ny) ? ca + 2 * a.nx - sz : ca + 2 * a.nx;
    const long dl = (x0 == 0) ? (long)a.nx - 1 : -1;                // column x0 - 1
    const long dr = (x0 + 2 == a.nx) ? 2 - (long)a.nx : 2;          // column x0 + 2
    // x neighbours of a pair: column x0 - 1 is the previous lane's second value, x0 + 2 the
    // next lane's first
    auto nb_l = [&](const P2& v, int c, size_t q) -> T {
      const T s = lane_from<T>(v.y, src_l);
      return edge_l ? F.raw(c, q + dl) : s;
    };
    auto nb_r = [&](const P2& v, int c, size_t q) -> T {
      const T s = lane_from<T>(v.x, src_r);
      return edge_r ? F.raw(c, q + dr) : s;
    };
    const size_t pm = (size_t)(z0 == 0 ? a.nz - 1 : z0 - 1) * sz;
    const size_t p0 = (size_t)z0 * sz;
    // S33, S23, S13 (slots 2, 3, 4) of planes z - 1 and z, rows a and b
    P2 a2m = F.raw2(2, pm + ca), a3m = F.raw2(3, pm + ca), a4m = F.raw2(4, pm + ca);
    P2 b2m = F.raw2(2, pm + cb), b3m = F.raw2(3, pm + cb), b4m = F.raw2(4, pm + cb);
    P2 a2c = F.raw2(2, p0 + ca), a3c = F.raw2(3, p0 + ca), a4c = F.raw2(4, p0 + ca);
    P2 b2c = F.raw2(2, p0 + cb), b3c = F.raw2(3, p0 + cb), b4c = F.raw2(4, p0 + cb);
    // one plane step: S11, S22, S12 of rows a and b; S12, S22, S23 of the outer rows y - 1 and
    // y + 2; S33, S23, S13 of rows a and b on the next plane.  FP32 fields load the step after
    // next while the current one is evaluated.
    auto load_step = [&](int z, P2* v) {
      const size_t p = (size_t)z * sz;
      const size_t pn = (size_t)(z + 1 == a.nz ? 0 : z + 1) * sz;
      v[0] = F.raw2(0, p + ca); v[1] = F.raw2(1, p + ca); v[2] = F.raw2(5, p + ca);
      v[3] = F.raw2(0, p + cb); v[4] = F.raw2(1, p + cb); v[5] = F.raw2(5, p + cb);
      v[6] = F.raw2(5, p + ym); v[7] = F.raw2(1, p + ym); v[8] = F.raw2(3, p + ym);
      v[9] = F.raw2(5, p + yq); v[10] = F.raw2(1, p + yq); v[11] = F.raw2(3, p + yq);
      v[12] = F.raw2(2, pn + ca); v[13] = F.raw2(3, pn + ca); v[14] = F.raw2(4, pn + ca);
      v[15] = F.raw2(2, pn + cb); v[16] = F.raw2(3, pn + cb); v[17] = F.raw2(4, pn + cb);
    };
    constexpr bool kAhead = sizeof(T) == 4;     // (FP64 only in use: no look-ahead)
    P2 cur[18], nxt[18];
    load_step(z0, cur);
    for (int z = z0; z < z1; ++z) {
      const size_t p = (size_t)z * sz;
      if (kAhead) {
        if (z + 1 < z1) load_step(z + 1, nxt);
      } else if (z > z0) {
        load_step(z, cur);
      }
      const size_t qa = p + ca, qb = p + cb;
      const P2 a0 = cur[0], a1 = cur[1], a5 = cur[2], b0 = cur[3], b1 = cur[4], b5 = cur[5];
      const P2 a2p = cur[12], a3p = cur[13], a4p = cur[14], b2p = cur[15], b3p = cur[16], b4p = cur[17];
      // x neighbours of S11, S12 (rows a, b; this plane) and S13 (rows a, b; this plane)
      const double a0l = nb_l(a0, 0, qa), a0r = nb_r(a0, 0, qa), b0l = nb_l(b0, 0, qb), b0r = nb_r(b0, 0, qb);
      const double a5l = nb_l(a5, 5, qa), a5r = nb_r(a5, 5, qa), b5l = nb_l(b5, 5, qb), b5r = nb_r(b5, 5, qb);
      const double a4l = nb_l(a4c, 4, qa), a4r = nb_r(a4c, 4, qa), b4l = nb_l(b4c, 4, qb), b4r = nb_r(b4c, 4, qb);
      auto D = [](T v) { return (double)v; };
      double r[2][2][3];      // [column][row a, b][component]
      // column x0: x neighbours x0 + 1 (the pair's second value) and x0 - 1
      r[0][0][0] = ((D(a0.y) - a0l) + (D(b5.x) - D(cur[6].x)) + (D(a4p.x) - D(a4m.x))) * a.inv2h;
      r[0][0][1] = ((D(a5.y) - a5l) + (D(b1.x) - D(cur[7].x)) + (D(a3p.x) - D(a3m.x))) * a.inv2h;
      r[0][0][2] = ((D(a4c.y) - a4l) + (D(b3c.x) - D(cur[8].x)) + (D(a2p.x) - D(a2m.x))) * a.inv2h;
      r[0][1][0] = ((D(b0.y) - b0l) + (D(cur[9].x) - D(a5.x)) + (D(b4p.x) - D(b4m.x))) * a.inv2h;
      r[0][1][1] = ((D(b5.y) - b5l) + (D(cur[10].x) - D(a1.x)) + (D(b3p.x) - D(b3m.x))) * a.inv2h;
      r[0][1][2] = ((D(b4c.y) - b4l) + (D(cur[11].x) - D(a3c.x)) + (D(b2p.x) - D(b2m.x))) * a.inv2h;
      // column x0 + 1: x neighbours x0 + 2 and x0 (the pair's first value)
      r[1][0][0] = ((a0r - D(a0.x)) + (D(b5.y) - D(cur[6].y)) + (D(a4p.y) - D(a4m.y))) * a.inv2h;
      r[1][0][1] = ((a5r - D(a5.x)) + (D(b1.y) - D(cur[7].y)) + (D(a3p.y) - D(a3m.y))) * a.inv2h;
      r[1][0][2] = ((a4r - D(a4c.x)) + (D(b3c.y) - D(cur[8].y)) + (D(a2p.y) - D(a2m.y))) * a.inv2h;
      r[1][1][0] = ((b0r - D(b0.x)) + (D(cur[9].y) - D(a5.y)) + (D(b4p.y) - D(b4m.y))) * a.inv2h;
      r[1][1][1] = ((b5r - D(b5.x)) + (D(cur[10].y) - D(a1.y)) + (D(b3p.y) - D(b3m.y))) * a.inv2h;
      r[1][1][2] = ((b4r - D(b4c.x)) + (D(cur[11].y) - D(a3c.y)) + (D(b2p.y) - D(b2m.y))) * a.inv2h;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double ma = r[k][0][0] * r[k][0][0] + r[k][0][1] * r[k][0][1] + r[k][0][2] * r[k][0][2];
        const double mb = r[k][1][0] * r[k][1][0] + r[k][1][1] * r[k][1][1] + r[k][1][2] * r[k][1][2];
        acc[0] += ma + mb;
        acc[1] = fmax(acc[1], fmax(ma, mb));
      }
      {
        // component statistics of the four voxels (slots 0 .. 5), about the shifts
        const double v[6][4] = {{D(a0.x), D(a0.y), D(b0.x), D(b0.y)},     {D(a1.x), D(a1.y), D(b1.x), D(b1.y)},
                                {D(a2c.x), D(a2c.y), D(b2c.x), D(b2c.y)}, {D(a3c.x), D(a3c.y), D(b3c.x), D(b3c.y)},
                                {D(a4c.x), D(a4c.y), D(b4c.x), D(b4c.y)}, {D(a5.x), D(a5.y), D(b5.x), D(b5.y)}};
        const double shv[6] = {sh0, sh1, sh2, sh3, sh4, sh5};
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double d = v[c][k] - shv[c];
            acc[2 + c] += d;
            acc[8 + c] += d * d;
          }
      }
      if (div) {
        T* o = div + (size_t)b * 3 * M;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          *reinterpret_cast<P2*>(o + c * M + qa) = P2{(T)r[0][0][c], (T)r[1][0][c]};
          *reinterpret_cast<P2*>(o + c * M + qb) = P2{(T)r[0][1][c], (T)r[1][1][c]};
        }
      }
      if (kAhead) {
#pragma unroll
        for (int k = 0; k < 18; ++k) cur[k] = nxt[k];
      }
      a2m = a2c; a3m = a3c; a4m = a4c;
      a2c = a2p; a3c = a3p; a4c = a4p;
      b2m = b2c; b3m = b3c; b4m = b4c;
      b2c = b2p; b3c = b3p; b4c = b4p;
    }
  }
  block_reduce_record(acc, sh);
  if (threadIdx.x == 0) {
    double* pp = partials + ((size_t)b * gridDim.x + blockIdx.x) * kRedWidth;
#pragma unroll
    for (int k = 0; k < kRedWidth; ++k) pp[k] = acc[k];
  }
}

struct DsArgs {
  int nx, ny, nz;
  size_t div_field, div_comp;
};

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_div_stats(const T* __restrict__ div, const T* __restrict__ S,
                                                           double* __restrict__ partials, DsArgs a) {
  __shared__ double sh[kRedWidth * kRedThreads];
  const int b = blockIdx.y;
  const size_t M = (size_t)a.nx * a.ny * a.nz;
  const T* F = S + (size_t)b * 6 * M;
  const T* R = div + (size_t)b * a.div_field;
  double acc[kRedWidth];
#pragma unroll
  for (int k = 0; k < kRedWidth; ++k) acc[k] = 0.0;
  double shift[6];                       // sums about the field's first voxel (see k_div_ddo)
#pragma unroll
  for (int c = 0; c < 6; ++c) shift[c] = uniform_f64((double)F[c * M]);
  for (size_t v = (size_t)blockIdx.x * kRedThreads + threadIdx.x; v < M; v += (size_t)gridDim.x * kRedThreads) {
    const double r0 = R[v], r1 = R[a.div_comp + v], r2 = R[2 * a.div_comp + v];
    const double m2 = r0 * r0 + r1 * r1 + r2 * r2;
    acc[0] += m2;
    acc[1] = fmax(acc[1], m2);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double s = (double)F[c * M + v] - shift[c];
      acc[2 + c] += s;
      acc[8 + c] += s * s;
    }
  }
  block_reduce_record(acc, sh);
  if (threadIdx.x == 0) {
    double* pp = partials + ((size_t)b * gridDim.x + blockIdx.x) * kRedWidth;
#pragma unroll
    for (int k = 0; k < kRedWidth; ++k) pp[k] = acc[k];
  }
}

// Field b's record from its nblk partial records (same order whatever the caller).
__device__ __forceinline__ void reduce_field_record(const double* __restrict__ partials, int nblk, int b,
                                                    double* acc, double* sh) {
#pragma unroll
  for (int k = 0; k < kRedWidth; ++k) acc[k] = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kRedThreads) {
    const double* pp = partials + ((size_t)b * nblk + i) * kRedWidth;
#pragma unroll
    for (int k = 0; k < kRedWidth; ++k) acc[k] = (k == 1) ? fmax(acc[k], pp[k]) : acc[k] + pp[k];
  }
  block_reduce_record(acc, sh);
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* __restrict__ partials, int nblk,
                                                              double* __restrict__ out) {
  __shared__ double sh[kRedWidth * kRedThreads];
  const int b = blockIdx.x;
  double acc[kRedWidth];
  reduce_field_record(partials, nblk, b, acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kRedWidth; ++k) out[(size_t)b * kRedWidth + k] = acc[k];
  }
}

// The same reduction, finished on the device: norms[b] = (l2, max, rel) with
// rel = l2 / (smax * ||S - c0||_F), ||S - c0||_F^2 = sum_c w_c (sum d_c^2 - (sum d_c)^2 / M).
__global__ __launch_bounds__(kRedThreads) void k_reduce_norms(const double* __restrict__ partials, int nblk,
                                                              double inv_m, double smax, double* __restrict__ norms) {
  __shared__ double sh[kRedWidth * kRedThreads];
  const int b = blockIdx.x;
  double acc[kRedWidth];
  reduce_field_record(partials, nblk, b, acc, sh);
  if (threadIdx.x == 0) {
    const double w[6] = {1, 1, 1, 2, 2, 2};
    double dev2 = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) dev2 += w[c] * (acc[8 + c] - acc[2 + c] * acc[2 + c] * inv_m);
    const double l2 = sqrt(acc[0]);
    const double denom = smax * sqrt(fmax(dev2, 0.0));
    norms[3 * b + 0] = l2;
    norms[3 * b + 1] = sqrt(acc[1]);
    norms[3 * b + 2] = denom > 0.0 ? l2 / denom : 0.0;
  }
}

// Scratch of the allocation-free residual (eq_residual_noalloc): the partial records of up
// to kNoAllocFields fields of at most kRedBlocks workgroups each, 7.3 MB held by every device
// the library runs on until the process ends.  Host code never passes this name to a kernel:
// it takes the device address from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) double scratch[(size_t)kNoAllocFields * kRedBlocks * kRedWidth];

template <typename T>
__global__ void k_check_finite(const T* __restrict__ p, size_t n, int* flag) {
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    bad |= !isfinite(p[i]);
  if (bad) atomicOr(flag, 1);
}

__global__ void k_fill_int(int* p, int n, int value) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = value;
}

template <typename T>
size_t csize() { return sizeof(cplx<T>); }

// Compile-time radix schedules on (default) or off (EQ_CT=0, for comparisons).
bool ct_enabled() {
  const char* e = std::getenv("EQ_CT");
  return !(e && e[0] == '0');
}

// Issue a register-engine launch: a compile-time schedule when one matches the
// axis's radix list, else the run-time schedule.
template <typename T>
void dispatch_fast(const FastArgs<T>& a) {
  if (ct_enabled() && (ct_launch_pow2<T>(a) || ct_launch_mixed<T>(a))) return;
  // unreachable: radix-4 plans (E = 4, 12, 20) exist only where the x6 schedules above serve
  // them (the planner checks), and no run-time engine has these E
  if (a.E == 4 || a.E == 12 || a.E == 20) return;
  switch (a.E) {
    case 8: launch_with<T, RtFft<8>>(a); break;
    case 16: launch_with<T, RtFft<16>>(a); break;
    case 24: launch_with<T, RtFft<24>>(a); break;
    default: launch_with<T, RtFft<40>>(a); break;
  }
}

int round_threads(int t) { return t < 64 ? 64 : ((t + 63) / 64) * 64; }

int largest_pow2_divisor_le(int n, int cap) {
  int t = 1;
  while (t * 2 <= cap && n % (t * 2) == 0) t *= 2;
  return t;
}

}  // namespace

// ------------------------------------------------------------- shapes ------

// The six-component x kernel keeps 6 * E complex values per lane: used for E = 8 in
// FP32 (96 VGPRs of data); EQ_X6=0/1 overrides (FP64 E = 8 doubles that).
template <typename T>
bool use_x6(const AxisFft& ax) {
  // needs a compile-time radix-8 schedule (the powers of two 32 .. 512, eq_sched_pow2.hip)
  const int n = ax.d.n;
  if (!ax.fast || (ax.E != 8 && ax.E != 4) || n < 32 || n > 512 || (n & (n - 1)) != 0 || !ct_enabled()) return false;
  const char* e = std::getenv("EQ_X6");
  if (e) return e[0] == '1';
  return sizeof(T) == 4;
}
bool use_x6_eb(const AxisFft& ax, int eb) { return eb == 8 ? use_x6<float>(ax) : use_x6<double>(ax); }
// The half-split six-component kernel (three rows per lane): needs an even E, P = nx / E
// dividing the 32 lanes of a wavefront half (k_x6s_r) or P = 64, one wavefront per
// component triple (k_x6w_r), and a compile-time schedule for the axis.
// Default for E <= 16 (the power-of-two schedules), where halving the registers per lane
// measured 10-20 % faster; the 3/5-smooth schedules (E = 24, 40) keep their line kernel.
template <typename T>
bool x6s_schedule(const AxisFft& ax) {
  FastArgs<T> f;
  f.kind = KK_X6S;
  f.n = ax.d.n;
  f.E = ax.E;
  f.d = ax.d;
  f.dry = true;
  return ct_launch_pow2<T>(f) || ct_launch_mixed<T>(f);
}
bool x_split(const AxisFft& ax, int eb, const Tune& tn) {
  // E = 12 and 20 (radix 4 with a factor 3 or 5) exist only for the split kernel, so it is their default
  if (tn.xsplit == 1 || (tn.xsplit == 0 && ax.E > 16 && ax.E != 20)) return false;
  if (!ax.fast || !ct_enabled() || ax.E % 2 != 0) return false;
  const int P = ax.d.n / ax.E;
  if (P < 1 || (P > 32 && P != 64) || (P <= 32 && 32 % P != 0)) return false;
  return eb == 8 ? x6s_schedule<float>(ax) : x6s_schedule<double>(ax);
}
bool x6_radix4_available(int nx, bool fp64) {
  if (fp64) return false;
  AxisFft ax{};
  ax.d.n = nx;
  ax.E = 4;
  ax.fast = true;
  if (use_x6<float>(ax)) return true;          // powers of two: the six-component kernels, E = 4
  // 3- or 5-smooth: the split kernel on a radix-4 schedule (E = 12 or 20), where one exists
  int m = nx, a = 0, b = 0, c = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  while (m % 5 == 0) { m /= 5; ++c; }
  if (m != 1 || a < 3 || (b > 0) == (c > 0)) return false;
  ax.E = b > 0 ? 12 : 20;
  int k = 0;
  for (int i = 0; i < a / 2; ++i) ax.d.r[k++] = 4;
  if (a % 2) ax.d.r[k++] = 2;
  for (int i = 0; i < b; ++i) ax.d.r[k++] = 3;
  for (int i = 0; i < c; ++i) ax.d.r[k++] = 5;
  ax.d.nst = k;
  const int P = nx / ax.E;
  return ct_enabled() && P >= 1 && P <= 32 && 32 % P == 0 && x6s_schedule<float>(ax);
}
// Register-engine shapes aim at ~256 threads per workgroup (several workgroups per
// CU so load, transform and store phases of different workgroups overlap) with
// tiles at least 128 bytes wide along x.

int pick_tx_y(const Geom& g, const AxisFft& ay, int eb, const Tune& tn) {
  if (tn.tx_y > 0) return tn.tx_y;
  const int P = g.ny / ay.E;
  if (ay.fast) {
    const int min_tx = 128 / eb;
    int want = 256 / P;
    if (want < min_tx) want = min_tx;
    int tx = largest_pow2_divisor_le(g.nx, want > 64 ? 64 : want);
    while (tx > 1 && (tx * P > kMaxFastThreads || (size_t)tx * g.ny * eb > kLdsPreferred)) tx >>= 1;
    return tx;
  }
  int tx = 64;
  while (tx > 1 && (g.nx % tx != 0 || tx * P > kMaxThreads || (size_t)tx * g.ny * eb > kLdsPreferred)) tx >>= 1;
  return tx;
}

int pick_tx_z(const Geom& g, const AxisFft& az, int eb, const Tune& tn) {
  if (tn.tx_z > 0) return tn.tx_z;
  const int P = g.nz / az.E;
  if (az.fast) {
    const int min_np = 128 / eb;
    int want = 256 / P;
    if (want < min_np) want = min_np;
    int tx = 2 * largest_pow2_divisor_le(g.nx / 2, want > 64 ? 64 : want);
    while (tx > 2 && ((tx / 2) * P > kMaxFastThreads || (size_t)(tx / 2) * g.nz * eb > kLdsPreferred)) tx >>= 1;
    return tx;
  }
  int tx = 128;
  while (tx > 2 && (g.nx % tx != 0 || (tx / 2) * P > kMaxThreads || (size_t)(tx / 2) * g.nz * eb > kLdsPreferred))
    tx >>= 1;
  return tx;
}

int pick_rw_x(const Geom& g, const AxisFft& ax, int eb, const Tune& tn) {
  if (tn.rw_x > 0) return tn.rw_x;
  const int P = g.nx / ax.E;
  if (x_split(ax, eb, tn)) {
    // two wavefronts per workgroup (measured best), one where LDS would pass 64 KiB
    const size_t row_lds = (size_t)6 * (g.nx + (g.nx >> kX6Skew) + 1) * eb;
    return (size_t)(64 / P) * row_lds <= kLdsPreferred ? 64 / P : 32 / P;
  }
  if (use_x6_eb(ax, eb)) {
    // one thread per (row, p); about 64 threads (one wavefront) per workgroup measured best
    int rw = 64 / P;
    if (rw < 1) rw = 1;
    const int ls = g.nx + (g.nx >> kX6Skew) + 1;
    while (rw > 1 && (rw * P > kMaxFastThreads || (size_t)3 * rw * ls * eb > kLdsPreferred)) --rw;
    return rw;
  }
  if (ax.fast) {
    // one line per thread group: about 128 threads per workgroup (several rows when lines are short)
    const int ls = g.nx + (g.nx >> kSkew) + 1;
    int rw = 128 / (6 * P);
    if (rw < 1) rw = 1;
    while (rw > 1 && (6 * rw * P > kMaxFastThreads || (size_t)6 * rw * ls * eb > kLdsPreferred)) --rw;
    return rw;
  }
  int rw = 16;
  while (rw > 1 && (6 * rw * P > kMaxThreads || (size_t)6 * rw * (g.nx + 1) * eb > kLdsPreferred)) --rw;
  return rw;
}

int max_threads(const AxisFft& ax) { return ax.fast ? kMaxFastThreads : kMaxThreads; }
int x_threads_per_row(const AxisFft& ax, int eb, const Tune& tn) {
  return (x_split(ax, eb, tn) ? 2 : use_x6_eb(ax, eb) ? 1 : 6) * (ax.d.n / ax.E);
}

size_t lds_y(const Geom& g, const AxisFft& ay, int eb, const Tune& tn) {
  return (size_t)pick_tx_y(g, ay, eb, tn) * g.ny * eb;
}
size_t lds_z(const Geom& g, const AxisFft& az, int eb, const Tune& tn) {
  return (size_t)(pick_tx_z(g, az, eb, tn) / 2) * g.nz * eb;
}
size_t lds_x(const Geom& g, const AxisFft& ax, int eb, const Tune& tn) {
  if (x_split(ax, eb, tn)) {
    // six lines per row for every row the (whole-wavefront) workgroup covers
    const int P = g.nx / ax.E;
    const int rows = round_threads(2 * P * pick_rw_x(g, ax, eb, tn)) / (2 * P);
    return (size_t)6 * rows * (g.nx + (g.nx >> kX6Skew) + 1) * eb;
  }
  const bool six = use_x6_eb(ax, eb);
  const int ls = !ax.fast ? g.nx + 1 : g.nx + (g.nx >> (six ? kX6Skew : kSkew)) + 1;
  const int lines = six ? 3 : 6;     // the six-component kernel transforms three rows at a time
  return (size_t)lines * pick_rw_x(g, ax, eb, tn) * ls * eb;
}

// ----------------------------------------------------------- launchers -----

hipError_t launch_tables(const Geom& g, int op, double h, double* sym, double2* tw64, float2* tw32, hipStream_t s) {
  const int total = g.nx + g.ny + g.nz;
  hipLaunchKernelGGL(k_tables, dim3((total + 255) / 256), dim3(256), 0, s, g.nx, g.ny, g.nz, op, h, sym, tw64, tw32);
  return hipGetLastError();
}

#define EQ_GEN_E_SWITCH(E_, BODY)  \
  switch (E_) {                    \
    case 8: { constexpr int EE = 8; BODY; } break;   \
    case 4: { constexpr int EE = 4; BODY; } break;   \
    default: { constexpr int EE = 2; BODY; } break;  \
  }

template <typename T>
FastArgs<T> fast_args(KernelKind kind, const AxisFft& ax, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                      const cplx<T>* tw) {
  FastArgs<T> f;
  f.kind = kind;
  f.n = ax.d.n;
  f.E = ax.E;
  f.grid = grid;
  f.block = block;
  f.lds = lds;
  f.s = s;
  f.d = ax.d;
  f.tw = tw;
  return f;
}

template <typename T>
hipError_t launch_z_r2c(const T* in, cplx<T>* W, const Geom& g, const AxisFft& az, const cplx<T>* tw_z,
                        const Tune& tn, hipStream_t s, const Embed& e) {
  const int eb = (int)csize<T>();
  const int tx = pick_tx_z(g, az, eb, tn);
  ZArgs a{g.nx, g.ny, g.nz, tx, e};
  const size_t lds = lds_z(g, az, eb, tn);
  const dim3 grid((unsigned)((size_t)(g.nx / tx) * g.ny * g.batch * 6));
  const int P = g.nz / az.E;
  if (az.fast) {
    FastArgs<T> f = fast_args<T>(KK_Z_R2C, az, grid, dim3((tx / 2) * P), lds, s, tw_z);
    f.in = in;
    f.W = W;
    f.za = a;
    dispatch_fast<T>(f);
  } else {
    const dim3 block(round_threads((tx / 2) * P));
    EQ_GEN_E_SWITCH(az.E, hipLaunchKernelGGL((k_z_r2c_g<T, EE>), grid, block, lds, s, in, W, a, az.d, tw_z));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_y(cplx<T>* W, const Geom& g, int pl0, int npl, int ncomp, const AxisFft& ay, const cplx<T>* tw_y,
                    bool inv, const Tune& tn, hipStream_t s) {
  const int eb = (int)csize<T>();
  const int tx = pick_tx_y(g, ay, eb, tn);
  YArgs a{g.nx, g.ny, g.nzh, ncomp, tx, pl0, npl};
  const size_t lds = lds_y(g, ay, eb, tn);
  const dim3 grid((unsigned)((size_t)(g.nx / tx) * npl * ncomp));
  const int P = g.ny / ay.E;
  if (ay.fast) {
    FastArgs<T> f = fast_args<T>(inv ? KK_Y_INV : KK_Y_FWD, ay, grid, dim3(tx * P), lds, s, tw_y);
    f.W = W;
    f.ya = a;
    dispatch_fast<T>(f);
  } else {
    const dim3 block(round_threads(tx * P));
    if (inv) { EQ_GEN_E_SWITCH(ay.E, hipLaunchKernelGGL((k_y_g<T, EE, true>), grid, block, lds, s, W, a, ay.d, tw_y)); }
    else { EQ_GEN_E_SWITCH(ay.E, hipLaunchKernelGGL((k_y_g<T, EE, false>), grid, block, lds, s, W, a, ay.d, tw_y)); }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_x(cplx<T>* W, const Geom& g, int pl0, int npl, int mode, const AxisFft& ax, const cplx<T>* tw_x,
                    const double* sym, const Tune& tn, hipStream_t s, double h) {
  const int eb = (int)csize<T>();
  const int rw = pick_rw_x(g, ax, eb, tn);
  const int rows = npl * g.ny;
  XArgs a{g.nx, g.ny, g.nzh, pl0, rows, rw, mode, h};
  const size_t lds = lds_x(g, ax, eb, tn);
  const dim3 grid((unsigned)((rows + rw - 1) / rw));
  const int P = g.nx / ax.E;
  if (ax.fast && x_split(ax, eb, tn)) {
    FastArgs<T> f = fast_args<T>(KK_X6S, ax, grid, dim3(round_threads(2 * P * rw)), lds, s, tw_x);
    f.W = W;
    f.xa = a;
    f.sym = sym;
    dispatch_fast<T>(f);
  } else if (ax.fast) {
    const bool six = use_x6<T>(ax);
    FastArgs<T> f = fast_args<T>(six ? KK_X6 : KK_X, ax, grid, dim3((six ? 1 : 6) * rw * P), lds, s, tw_x);
    f.W = W;
    f.xa = a;
    f.sym = sym;
    dispatch_fast<T>(f);
  } else {
    const dim3 block(round_threads(6 * rw * P));
    EQ_GEN_E_SWITCH(ax.E, hipLaunchKernelGGL((k_x_g<T, EE>), grid, block, lds, s, W, a, ax.d, tw_x, sym));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_z_c2r(const cplx<T>* W, T* out, size_t out_field, size_t out_comp, const T* in, T* removed,
                        int ncomp, const Geom& g, const AxisFft& az, const cplx<T>* tw_z, const Tune& tn,
                        hipStream_t s, const Embed& e) {
  const int eb = (int)csize<T>();
  const int tx = pick_tx_z(g, az, eb, tn);
  ZcArgs a{g.nx, g.ny, g.nz, tx, ncomp, out_field, out_comp, e};
  const size_t lds = lds_z(g, az, eb, tn);
  const dim3 grid((unsigned)((size_t)(g.nx / tx) * g.ny * ncomp * g.batch));
  const T scale = (T)(1.0 / ((double)g.nx * (double)g.ny * (double)g.nz));
  const int P = g.nz / az.E;
  if (az.fast) {
    FastArgs<T> f = fast_args<T>(KK_Z_C2R, az, grid, dim3((tx / 2) * P), lds, s, tw_z);
    f.Wc = W;
    f.out = out;
    f.in = in;
    f.removed = removed;
    f.zca = a;
    f.scale = scale;
    dispatch_fast<T>(f);
  } else {
    const dim3 block(round_threads((tx / 2) * P));
    EQ_GEN_E_SWITCH(az.E, hipLaunchKernelGGL((k_z_c2r_g<T, EE>), grid, block, lds, s, W, out, in, removed, a, az.d,
                                             tw_z, scale));
  }
  return hipGetLastError();
}

// Buffer loads need each component's byte range below 2^31 (EQ_DDO_BUF=0 forces plain
// loads, so that both paths can be compared on small grids).
template <typename T>
bool div_ddo_buf(const Geom& g) {
  const char* e = std::getenv("EQ_DDO_BUF");
  if (e && e[0] == '0') return false;
  return (double)g.nx * g.ny * g.nz * sizeof(T) < 2147483648.0;
}

// The two-column kernel serves FP64 fields with nx a multiple of 128 (one wavefront spans
// 128 columns).
template <typename T>
bool div_ddo_pairs(const Geom& g) {
  return sizeof(T) == 8 && g.nx % 128 == 0;
}

// Workgroups of the DDO divergence kernel the device holds at once (CUs x resident
// workgroups per CU).
template <typename T, bool BUF, bool PAIRS>
int div_ddo_capacity() {
  static const int cap = [] {
    int dev = 0, cus = 0, per = 0;
    const void* k = nullptr;
    if constexpr (PAIRS) k = reinterpret_cast<const void*>(&k_div_ddo2<T, BUF>);
    else k = reinterpret_cast<const void*>(&k_div_ddo<T, BUF>);
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kRedThreads, 0) != hipSuccess)
      return 0;
    return cus * per;
  }();
  return cap;
}
template <typename T>
int div_ddo_cap(const Geom& g) {
  if constexpr (sizeof(T) == 8) {
    if (div_ddo_pairs<T>(g))
      return div_ddo_buf<T>(g) ? div_ddo_capacity<T, true, true>() : div_ddo_capacity<T, false, true>();
  }
  return div_ddo_buf<T>(g) ? div_ddo_capacity<T, true, false>() : div_ddo_capacity<T, false, false>();
}

// z chunks per work item: the count that wastes least of the resident capacity G for one
// field (the fewest items on ties), at least 8 planes per march where possible.
static int div_ddo_chunks(int tiles, int nz, int G) {
  const int zmax = nz >= 16 ? nz / 8 : 1;
  double best = -1.0;
  int zc = 1;
  for (int c = 1; c <= zmax; ++c) {
    const long items = (long)tiles * c;
    const long grid = items < G ? items : G;
    const long rounds = (items + grid - 1) / grid;
    const double eff = ((double)tiles * nz / G) / ((double)rounds * ((nz + c - 1) / c));
    if (eff > best + 1e-9) { best = eff; zc = c; }
  }
  return zc;
}

// Two-column shape: tiles of 128 columns by 8 rows (the last row group may be short).
static DvArgs div_ddo2_shape(const Geom& g, int nblk_max, double h, int cap) {
  DvArgs a{};
  a.nx = g.nx; a.ny = g.ny; a.nz = g.nz;
  a.tiles_x = g.nx / 128;
  a.tiles = a.tiles_x * ((g.ny + 7) / 8);
  a.zc = div_ddo_chunks(a.tiles, g.nz, cap > 0 && cap < nblk_max ? cap : nblk_max);
  a.inv2h = 0.5 / h;
  return a;
}

// Tiles of tx x (2 ty) columns, z chunks per column; a work item is (tile, z chunk), and the
// grid of a field (at most the device's resident capacity, at most nblk_max) loops over the
// items.  The kernel lasts (rounds) x (planes per item), so the chunk count is the one that
// wastes least of the resident capacity for one field (the fewest items on ties).  The
// shape depends on the field, not on the batch, so a field's partial sums, and so its
// norms, come out the same alone or in a batch.
static DArgs div_ddo_shape(const Geom& g, int nblk_max, double h, int cap) {
  DArgs a{};
  a.nx = g.nx; a.ny = g.ny; a.nz = g.nz;
  // widest x tile that divides nx (full rows at 256): long row segments, x halo in-tile
  a.tx = 64;
  for (int t : {256, 128, 64, 32, 16, 8})
    if (g.nx % t == 0) { a.tx = t; break; }
  a.ty = kRedThreads / a.tx;                 // thread rows; each thread takes two grid rows
  a.tiles_x = (g.nx + a.tx - 1) / a.tx;
  a.tiles = a.tiles_x * ((g.ny + 2 * a.ty - 1) / (2 * a.ty));
  a.zc = div_ddo_chunks(a.tiles, g.nz, cap > 0 && cap < nblk_max ? cap : nblk_max);
  a.inv2h = 0.5 / h;
  return a;
}

int div_ddo_blocks(const Geom& g, int nblk_max, bool fp64) {
  const int cap = fp64 ? div_ddo_cap<double>(g) : div_ddo_cap<float>(g);
  const int G = cap > 0 && cap < nblk_max ? cap : nblk_max;
  long items;
  if (fp64 ? div_ddo_pairs<double>(g) : div_ddo_pairs<float>(g)) {
    const DvArgs a = div_ddo2_shape(g, nblk_max, 1.0, cap);
    items = (long)a.tiles * a.zc;
  } else {
    const DArgs a = div_ddo_shape(g, nblk_max, 1.0, cap);
    items = (long)a.tiles * a.zc;
  }
  return (int)(items < G ? items : G);
}

template <typename T>
hipError_t launch_div_ddo(const T* S, T* div_out, double* partials, int nblk_max, const Geom& g, double h, hipStream_t s) {
  const dim3 grid(div_ddo_blocks(g, nblk_max, sizeof(T) == 8), g.batch);
  if constexpr (sizeof(T) == 8) {
    if (div_ddo_pairs<T>(g)) {
      const DvArgs a = div_ddo2_shape(g, nblk_max, h, div_ddo_cap<T>(g));
      if (div_ddo_buf<T>(g))
        hipLaunchKernelGGL((k_div_ddo2<T, true>), grid, dim3(kRedThreads), 0, s, S, div_out, partials, a);
      else
        hipLaunchKernelGGL((k_div_ddo2<T, false>), grid, dim3(kRedThreads), 0, s, S, div_out, partials, a);
      return hipGetLastError();
    }
  }
  const DArgs a = div_ddo_shape(g, nblk_max, h, div_ddo_cap<T>(g));
  if (div_ddo_buf<T>(g))
    hipLaunchKernelGGL((k_div_ddo<T, true>), grid, dim3(kRedThreads), 0, s, S, div_out, partials, a);
  else
    hipLaunchKernelGGL((k_div_ddo<T, false>), grid, dim3(kRedThreads), 0, s, S, div_out, partials, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_div_stats(const T* div, size_t div_field, size_t div_comp, const T* S, double* partials, int nblk,
                            const Geom& g, hipStream_t s) {
  DsArgs a{g.nx, g.ny, g.nz, div_field, div_comp};
  hipLaunchKernelGGL((k_div_stats<T>), dim3(nblk, g.batch), dim3(kRedThreads), 0, s, div, S, partials, a);
  return hipGetLastError();
}

hipError_t launch_reduce_final(const double* partials, int nblk, int batch, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(batch), dim3(kRedThreads), 0, s, partials, nblk, out);
  return hipGetLastError();
}

hipError_t launch_reduce_norms(const double* partials, int nblk, int batch, double inv_m, double smax, double* norms,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_norms, dim3(batch), dim3(kRedThreads), 0, s, partials, nblk, inv_m, smax, norms);
  return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per device (each device
// holds its own copy of the array at its own address).
hipError_t noalloc_scratch(double** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* ptrs[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptrs[dev] = static_cast<double*>(p);
  }
  *out = ptrs[dev];
  return hipSuccess;
}

template <typename T>
hipError_t launch_check_finite(const T* in, size_t n, int* flag, hipStream_t s) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL((k_check_finite<T>), dim3((unsigned)blocks), dim3(256), 0, s, in, n, flag);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, p, n, value);
  return hipGetLastError();
}

// ------------------------------------------------------ instantiations -----

#define EQ_INSTANTIATE(T)                                                                                          \
  template hipError_t launch_z_r2c<T>(const T*, cplx<T>*, const Geom&, const AxisFft&, const cplx<T>*,           \
                                      const Tune&, hipStream_t, const Embed&);                                     \
  template hipError_t launch_y<T>(cplx<T>*, const Geom&, int, int, int, const AxisFft&, const cplx<T>*, bool,     \
                                  const Tune&, hipStream_t);                                                       \
  template hipError_t launch_x<T>(cplx<T>*, const Geom&, int, int, int, const AxisFft&, const cplx<T>*,          \
                                  const double*, const Tune&, hipStream_t, double);                                \
  template hipError_t launch_z_c2r<T>(const cplx<T>*, T*, size_t, size_t, const T*, T*, int, const Geom&,         \
                                      const AxisFft&, const cplx<T>*, const Tune&, hipStream_t, const Embed&);     \
  template hipError_t launch_div_ddo<T>(const T*, T*, double*, int, const Geom&, double, hipStream_t);           \
  template hipError_t launch_div_stats<T>(const T*, size_t, size_t, const T*, double*, int, const Geom&,         \
                                          hipStream_t);                                                            \
  template hipError_t launch_check_finite<T>(const T*, size_t, int*, hipStream_t);

EQ_INSTANTIATE(float)
EQ_INSTANTIATE(double)

}  // namespace eq
