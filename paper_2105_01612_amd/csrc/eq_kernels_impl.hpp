// eq_kernels_impl.hpp -- register-engine kernels of the projection, generic over the
// FFT policy (compile-time Sched<R...> or run-time RtFft<E>), and the launch helper
// that instantiates them.  Included by eq_kernels.hip (run-time policies) and by the
// eq_sched_*.hip translation units (compile-time schedules).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "eq_fft.hpp"
#include "eq_internal.hpp"

namespace eq {

constexpr int kMaxThreads = 1024;      // generic-engine workgroups
constexpr int kMaxFastThreads = 512;   // register-engine workgroups (up to 256 VGPRs per lane)
constexpr size_t kLdsPreferred = 64 * 1024;
constexpr int kX6Skew = 4;             // pad shift of the six-component x kernel's LDS lines

// ----------------------------------------------------- per-frequency ops ---

// 1/sqrt(x) in FP64: the hardware estimate refined by two Newton steps (each squares the
// relative error), for x in the range of |s|^2 of the h-free symbols, [1e-6, 30].
__device__ __forceinline__ double rsqrt_fp64(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * (1.5 - 0.5 * x * r * r);
  r = r * (1.5 - 0.5 * x * r * r);
  return r;
}

// Projection of one frequency: out = P A P, P = I - n n^T, n = s / |s| formed in FP64.
// The symbols passed here are h-free (s * h): the projection depends on the direction
// of s only.  Voigt slots: 0=11 1=22 2=33 3=23 4=13 5=12.
template <typename T>
__device__ __forceinline__ void project_one(cplx<T>* A /*6*/, double sx, double sy, double sz) {
  using C = cplx<T>;
  const double ss = sx * sx + sy * sy + sz * sz;
  if (!(ss > 0.0)) return;                                   // zero symbol: divergence-free, kept
  const double inv = rsqrt_fp64(ss);
  const T n0 = (T)(sx * inv), n1 = (T)(sy * inv), n2 = (T)(sz * inv);
  const C a00 = A[0], a11 = A[1], a22 = A[2], a12 = A[3], a02 = A[4], a01 = A[5];
  // b = A n
  C b0, b1, b2;
  b0.x = a00.x * n0 + a01.x * n1 + a02.x * n2;  b0.y = a00.y * n0 + a01.y * n1 + a02.y * n2;
  b1.x = a01.x * n0 + a11.x * n1 + a12.x * n2;  b1.y = a01.y * n0 + a11.y * n1 + a12.y * n2;
  b2.x = a02.x * n0 + a12.x * n1 + a22.x * n2;  b2.y = a02.y * n0 + a12.y * n1 + a22.y * n2;
  // c = n . b
  C cc;
  cc.x = n0 * b0.x + n1 * b1.x + n2 * b2.x;
  cc.y = n0 * b0.y + n1 * b1.y + n2 * b2.y;
  // out_ij = A_ij - n_i b_j - b_i n_j + c n_i n_j
  auto upd = [&](C aij, T ni, T nj, C bi, C bj) -> C {
    C o;
    const T nn = ni * nj;
    o.x = aij.x - ni * bj.x - nj * bi.x + cc.x * nn;
    o.y = aij.y - ni * bj.y - nj * bi.y + cc.y * nn;
    return o;
  };
  A[0] = upd(a00, n0, n0, b0, b0);
  A[1] = upd(a11, n1, n1, b1, b1);
  A[2] = upd(a22, n2, n2, b2, b2);
  A[3] = upd(a12, n1, n2, b1, b2);
  A[4] = upd(a02, n0, n2, b0, b2);
  A[5] = upd(a01, n0, n1, b0, b1);
}

// Divergence of one frequency: r_i = sum_j (i s_j) A_ij, written to slots 0..2.
template <typename T>
__device__ __forceinline__ void divergence_one(cplx<T>* A, double sx, double sy, double sz) {
  using C = cplx<T>;
  const T s0 = (T)sx, s1 = (T)sy, s2 = (T)sz;
  const int idx[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
  C r3[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const C p = A[idx[i][0]], q = A[idx[i][1]], w = A[idx[i][2]];
    const T re = s0 * p.x + s1 * q.x + s2 * w.x;
    const T im = s0 * p.y + s1 * q.y + s2 * w.y;
    r3[i] = mk<T>(-im, re);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) A[i] = r3[i];
}

// Potential of the removed part at one frequency.  The removed part is the symmetric
// gradient (grad y + grad y^T)/2 of Section 3.2; with the derivative symbol i s and
// n = s/|s|, b = A n, c = n.b, it is n b^T + b n^T - c n n^T = A - P A P, whose unique
// preimage with zero mean is y = i (c n - 2 b) / |s|.  Zero-symbol frequencies give 0.
// Symbols are h-free (unit spacing); |s| carries 1/h.  Result in slots 0..2.
template <typename T>
__device__ __forceinline__ void potential_one(cplx<T>* A, double sx, double sy, double sz, double h) {
  using C = cplx<T>;
  const double ss = sx * sx + sy * sy + sz * sz;
  if (!(ss > 0.0)) {
    A[0] = A[1] = A[2] = mk<T>((T)0, (T)0);
    return;
  }
  const double inv = rsqrt_fp64(ss);
  const T n0 = (T)(sx * inv), n1 = (T)(sy * inv), n2 = (T)(sz * inv), w = (T)(h * inv);
  const C a00 = A[0], a11 = A[1], a22 = A[2], a12 = A[3], a02 = A[4], a01 = A[5];
  C b0, b1, b2;
  b0.x = a00.x * n0 + a01.x * n1 + a02.x * n2;  b0.y = a00.y * n0 + a01.y * n1 + a02.y * n2;
  b1.x = a01.x * n0 + a11.x * n1 + a12.x * n2;  b1.y = a01.y * n0 + a11.y * n1 + a12.y * n2;
  b2.x = a02.x * n0 + a12.x * n1 + a22.x * n2;  b2.y = a02.y * n0 + a12.y * n1 + a22.y * n2;
  C cc;
  cc.x = n0 * b0.x + n1 * b1.x + n2 * b2.x;
  cc.y = n0 * b0.y + n1 * b1.y + n2 * b2.y;
  // i (c n_k - 2 b_k) w  =  (-(c.y n_k - 2 b_k.y) w, (c.x n_k - 2 b_k.x) w)
  auto pot = [&](T nk, C bk) -> C {
    return mk<T>(-(cc.y * nk - (T)2 * bk.y) * w, (cc.x * nk - (T)2 * bk.x) * w);
  };
  A[0] = pot(n0, b0);
  A[1] = pot(n1, b1);
  A[2] = pot(n2, b2);
}

// The three-output per-frequency operations of the x pass.
template <typename T>
__device__ __forceinline__ void vector_op(int mode, cplx<T>* A, double sx, double sy, double sz, double h) {
  if (mode & XM_DISP) potential_one<T>(A, sx, sy, sz, h);
  else divergence_one<T>(A, sx, sy, sz);
}

// Word 3 of a raw buffer resource on gfx9: 32-bit data format, no swizzle.  A buffer load
// takes a 32-bit byte offset (VGPR) plus a workgroup-uniform one (SGPR) against a base
// held in SGPRs, so per-lane addresses cost one register instead of two; reads outside
// the resource's range return 0.
constexpr int kBufWord3 = 0x00020000;

// Workgroups are dealt round-robin to the 8 XCDs (workgroup b to XCD b mod 8).  This
// bijection of [0, n) gives each XCD a contiguous run of work indices, so neighbouring
// work items share the lines of their XCD's L2: XCD x takes n/8 indices, one more when
// x < n mod 8, starting after those of the XCDs before it.
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// ------------------------------------------------------------ arguments ----

struct ZArgs {
  int nx, ny, nz, tx;      // tx: real x-columns per workgroup (even)
  Embed e;
};

struct ZcArgs {
  int nx, ny, nz, tx, ncomp;
  size_t out_field, out_comp;
  Embed e;
};

// Real column pair (x0, x0 + 1) of box row y inside an embedded sample: the element
// offsets of (z = 0, y - oy, x - ox) in the sample field, valid where ok0 / ok1.
struct EmbedPair {
  size_t off0, off1;
  size_t plane;      // ny0 * nx0
  bool ok0, ok1;
};
__device__ __forceinline__ EmbedPair embed_pair(const Embed& e, int y, int x0) {
  EmbedPair r;
  const int ys = y - e.oy, xs = x0 - e.ox;
  const bool row = ys >= 0 && ys < e.ny0;
  r.ok0 = row && xs >= 0 && xs < e.nx0;
  r.ok1 = row && xs + 1 >= 0 && xs + 1 < e.nx0;
  r.plane = (size_t)e.ny0 * e.nx0;
  const size_t base = row ? (size_t)ys * e.nx0 : 0;
  r.off0 = r.ok0 ? base + xs : 0;
  r.off1 = r.ok1 ? base + xs + 1 : 0;
  return r;
}

struct YArgs {
  int nx, ny, nzh, ncomp, tx, pl0, npl;
};

struct XArgs {
  int nx, ny, nzh, pl0, rows, rw, mode;   // rows = planes in range * ny
  double h;                               // voxel spacing (potential mode)
};

__device__ __forceinline__ size_t y_tile_base(const YArgs& a) {
  const int ntx = a.nx / a.tx;
  int bid = blockIdx.x;
  const int xt = bid % ntx; bid /= ntx;
  const int pll = bid % a.npl;
  const int c = bid / a.npl;
  const int pl = a.pl0 + pll;
  const int b = pl / a.nzh, kz = pl - b * a.nzh;
  return (((size_t)(b * 6 + c) * a.nzh + kz) * a.ny) * a.nx + (size_t)xt * a.tx;
}

__device__ __forceinline__ size_t x_row_base(const XArgs& a, int row, int c, int& kz, int& ky) {
  const int pl = a.pl0 + row / a.ny;
  ky = row - (row / a.ny) * a.ny;
  const int b = pl / a.nzh;
  kz = pl - b * a.nzh;
  return (((size_t)(b * 6 + c) * a.nzh + kz) * a.ny + ky) * a.nx;
}

// ------------------------------------------------------- z passes (r2c) ----

template <typename T, typename F>
__global__ __launch_bounds__(kMaxFastThreads) void k_z_r2c_r(const T* __restrict__ in, cplx<T>* __restrict__ W, ZArgs a,
                                                             FftDesc d, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int E = F::E;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int ntx = a.nx / a.tx;
  int bid = blockIdx.x;
  const int xt = bid % ntx; bid /= ntx;
  const int y = bid % a.ny;
  const int bc = bid / a.ny;                        // b * 6 + c
  const int np = a.tx >> 1;                         // complex lines (column pairs)
  const int nz = F::len(d), nzh = nz / 2 + 1, P = nz / E;
  const int line = threadIdx.x % np, p = threadIdx.x / np;
  const size_t plane = (size_t)a.ny * a.nx;
  C v[1][E];
  if (!a.e.on) {
    const T* src = in + (size_t)bc * nz * plane + (size_t)y * a.nx + (size_t)xt * a.tx + 2 * line;
#pragma unroll
    for (int i = 0; i < E; ++i) v[0][i] = *reinterpret_cast<const C*>(src + (size_t)(p + i * P) * plane);
  } else {
    // embedded sample: columns outside it are the zero-stress buffer
    const EmbedPair ep = embed_pair(a.e, y, xt * a.tx + 2 * line);
    const T* src = in + (size_t)bc * nz * ep.plane;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const size_t o = (size_t)(p + i * P) * ep.plane;
      v[0][i] = mk<T>(ep.ok0 ? src[o + ep.off0] : (T)0, ep.ok1 ? src[o + ep.off1] : (T)0);
    }
  }
  const LdsMap m{1, np, 0};
  F::template run<T, 1, false, true, false>(v, lds, m, line, 0, p, d, tw);
  // separate the two packed columns: A = (Z + conj Zm) / 2, B = (Z - conj Zm) / 2i;
  // thread (line, p) emits kz = p + i*P for the column pair `line`
  C* dst = W + (size_t)bc * nzh * plane + (size_t)y * a.nx + (size_t)xt * a.tx + 2 * line;
  const T half = (T)0.5;
  constexpr int NU = E / 2 + 1;
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    const int kz = p + i * P;
    if (kz < nzh) {
      const C Z = lds[kz * np + line];
      const C Zm = lds[(kz == 0 ? 0 : nz - kz) * np + line];
      C* o = dst + (size_t)kz * plane;
      o[0] = mk<T>((Z.x + Zm.x) * half, (Z.y - Zm.y) * half);
      o[1] = mk<T>((Z.y + Zm.y) * half, (Zm.x - Z.x) * half);
    }
  }
}

// ------------------------------------------------------- z passes (c2r) ----

template <typename T, typename F>
__global__ __launch_bounds__(kMaxFastThreads) void k_z_c2r_r(const cplx<T>* __restrict__ W, T* out, const T* in,
                                                             T* removed, ZcArgs a, FftDesc d,
                                                             const cplx<T>* __restrict__ tw, T scale) {
  using C = cplx<T>;
  constexpr int E = F::E;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int ntx = a.nx / a.tx;
  int bid = blockIdx.x;
  const int xt = bid % ntx; bid /= ntx;
  const int y = bid % a.ny; bid /= a.ny;
  const int c = bid % a.ncomp;
  const int b = bid / a.ncomp;
  const int np = a.tx >> 1;
  const int nz = F::len(d), nzh = nz / 2 + 1, nyq = nz / 2, P = nz / E;
  const int line = threadIdx.x % np, p = threadIdx.x / np;
  const size_t plane = (size_t)a.ny * a.nx;
  const C* src = W + ((size_t)(b * 6 + c) * nzh) * plane + (size_t)y * a.nx + (size_t)xt * a.tx;
  constexpr int NU = E / 2 + 1;
  constexpr int G = 8;                     // pairs loaded per group (bounds live registers)
  // pack the two columns of each pair into one complex line: Z = A + i B, Z(-k) = conj A + i conj B;
  // thread (line, p) reads kz = p + i*P of column pair `line`
  const C* col = src + 2 * line;
#pragma unroll
  for (int g0 = 0; g0 < NU; g0 += G) {
    C ab[G][2];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int kz = p + (g0 + i) * P;
      if (g0 + i < NU && kz < nzh) {
        const C* s = col + (size_t)kz * plane;
        ab[i][0] = s[0];
        ab[i][1] = s[1];
      }
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int kz = p + (g0 + i) * P;
      if (g0 + i < NU && kz < nzh) {
        C A = ab[i][0], B = ab[i][1];
        if (kz == 0 || kz == nyq) { A.y = (T)0; B.y = (T)0; }   // self-conjugate planes are real
        lds[kz * np + line] = mk<T>(A.x - B.y, A.y + B.x);
        if (kz > 0 && kz < nyq) lds[(nz - kz) * np + line] = mk<T>(A.x + B.y, B.x - A.y);
      }
    }
  }
  __syncthreads();
  // the input samples of the removed part are fetched before the transform, so their
  // latency hides behind it
  const size_t obase = (size_t)b * a.out_field + (size_t)c * a.out_comp + (size_t)y * a.nx + (size_t)xt * a.tx +
                       2 * line;
  C pre[E];
  if (removed && !a.e.on) {
#pragma unroll
    for (int i = 0; i < E; ++i) pre[i] = *reinterpret_cast<const C*>(in + obase + (size_t)(p + i * P) * plane);
  }
  C v[1][E];
  const LdsMap m{1, np, 0};
  F::template run<T, 1, true, false, true>(v, lds, m, line, 0, p, d, tw);
  if (a.e.on) {
    // embedded sample: write its voxels only, in sample coordinates
    const EmbedPair ep = embed_pair(a.e, y, xt * a.tx + 2 * line);
    const size_t sbase = (size_t)b * a.out_field + (size_t)c * a.out_comp;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const size_t o = sbase + (size_t)(p + i * P) * ep.plane;
      const T o0 = v[0][i].x * scale, o1 = v[0][i].y * scale;
      if (ep.ok0) {
        if (removed) removed[o + ep.off0] = in[o + ep.off0] - o0;
        out[o + ep.off0] = o0;
      }
      if (ep.ok1) {
        if (removed) removed[o + ep.off1] = in[o + ep.off1] - o1;
        out[o + ep.off1] = o1;
      }
    }
    return;
  }
  if (removed) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const C o = mk<T>(v[0][i].x * scale, v[0][i].y * scale);
      const size_t off = obase + (size_t)(p + i * P) * plane;
      *reinterpret_cast<C*>(removed + off) = mk<T>(pre[i].x - o.x, pre[i].y - o.y);
      *reinterpret_cast<C*>(out + off) = o;
    }
  } else {
#pragma unroll
    for (int i = 0; i < E; ++i)
      *reinterpret_cast<C*>(out + obase + (size_t)(p + i * P) * plane) =
          mk<T>(v[0][i].x * scale, v[0][i].y * scale);
  }
}

// ------------------------------------------------------------- y pass ------

template <typename T, typename F, bool INV>
__global__ __launch_bounds__(kMaxFastThreads) void k_y_r(cplx<T>* __restrict__ W, YArgs a, FftDesc d,
                                                         const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int E = F::E;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C* base = W + y_tile_base(a);
  const int tx = a.tx, P = F::len(d) / E;
  const int line = threadIdx.x % tx, p = threadIdx.x / tx;
  C* col = base + line;
  C v[1][E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[0][i] = col[(size_t)(p + i * P) * a.nx];
  const LdsMap m{1, tx, 0};
  F::template run<T, 1, INV, true, true>(v, lds, m, line, 0, p, d, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) col[(size_t)(p + i * P) * a.nx] = v[0][i];
}

// ------------------------------------------------------------- x pass ------

// One line per thread group: thread (line = c * rw + r, p); the six components of a
// frequency meet in LDS for the projection.
template <typename T, typename F>
__global__ __launch_bounds__(kMaxFastThreads) void k_x_r(cplx<T>* __restrict__ W, XArgs a, FftDesc d,
                                                         const cplx<T>* __restrict__ tw,
                                                         const double* __restrict__ sym) {
  using C = cplx<T>;
  constexpr int E = F::E;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int nx = F::len(d), rw = a.rw, P = nx / E;
  const int p = threadIdx.x % P, line = threadIdx.x / P;   // line = c * rw + r
  const int c = line / rw, r = line - c * rw;
  const int row0 = blockIdx.x * rw;
  const int nrows = min(rw, a.rows - row0);
  const bool valid = r < nrows;
  const int ncomp_out = (a.mode & (XM_DIV | XM_DISP)) ? 3 : 6;
  const bool active = c < ncomp_out;
  int kz, ky;
  const size_t base = valid ? x_row_base(a, row0 + r, c, kz, ky) + p : 0;
  C v[1][E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[0][i] = valid ? W[base + (size_t)i * P] : mk<T>((T)0, (T)0);
  const LdsMap m{nx + (nx >> kSkew) + 1, 1, kSkew};
  if (a.mode & XM_FWD) {
    F::template run<T, 1, false, true, false>(v, lds, m, line, 0, p, d, tw);
  } else {
#pragma unroll
    for (int i = 0; i < E; ++i) lds[m.at(line, p + i * P)] = v[0][i];
    __syncthreads();
  }
  if (a.mode & (XM_PROJ | XM_DIV | XM_DISP)) {
    const double* symx = sym;
    const double* symy = sym + nx;
    const double* symz = sym + nx + a.ny;
    const int nthr = 6 * rw * P;
    for (int rr = 0; rr < nrows; ++rr) {
      int qz, qy;
      (void)x_row_base(a, row0 + rr, 0, qz, qy);          // uniform across the workgroup
      const double sy = symy[qy], sz = symz[qz];
      for (int kx = threadIdx.x; kx < nx; kx += nthr) {
        C A[6];
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) A[cc] = lds[m.at(cc * rw + rr, kx)];
        if (a.mode & XM_PROJ) {
          project_one<T>(A, symx[kx], sy, sz);
#pragma unroll
          for (int cc = 0; cc < 6; ++cc) lds[m.at(cc * rw + rr, kx)] = A[cc];
        } else {
          vector_op<T>(a.mode, A, symx[kx], sy, sz, a.h);
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) lds[m.at(cc * rw + rr, kx)] = A[cc];
        }
      }
    }
    __syncthreads();
  }
  if (a.mode & XM_INV) {
    // every line takes the transform (and its barriers); lines of components a divergence
    // pass does not output hold finite spectra and are simply not stored
    F::template run<T, 1, true, false, true>(v, lds, m, line, 0, p, d, tw);
  } else {
#pragma unroll
    for (int i = 0; i < E; ++i) v[0][i] = lds[m.at(line, p + i * P)];
  }
  if (valid && active) {
#pragma unroll
    for (int i = 0; i < E; ++i) W[base + (size_t)i * P] = v[0][i];
  }
}

// Six-component x pass: thread (row r, p) owns elements p + i*P of all six component
// rows, so the projection (or divergence) of each of its frequencies runs in registers
// between the forward and inverse transforms.  The rows are transformed three
// components at a time, so LDS holds 3 * rw lines (twice the workgroups per CU).
template <typename T, typename F>
__global__ __launch_bounds__(kMaxFastThreads) void k_x6_r(cplx<T>* __restrict__ W, XArgs a, FftDesc d,
                                                          const cplx<T>* __restrict__ tw,
                                                          const double* __restrict__ sym) {
  using C = cplx<T>;
  constexpr int E = F::E;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int nx = F::len(d), P = nx / E;
  const int rw = a.rw;
  const int p = threadIdx.x % P, r = threadIdx.x / P;
  const int row0 = blockIdx.x * rw;
  const bool valid = r < min(rw, a.rows - row0);
  const size_t cstride = (size_t)a.nzh * a.ny * nx;      // between components of one field
  int kz = 0, ky = 0;
  const size_t base = valid ? x_row_base(a, row0 + r, 0, kz, ky) + p : 0;
  C v[6][E];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int i = 0; i < E; ++i) v[c][i] = valid ? W[base + c * cstride + (size_t)i * P] : mk<T>((T)0, (T)0);
  const LdsMap m{nx + (nx >> kX6Skew) + 1, 1, kX6Skew};
  if (a.mode & XM_FWD) {
    F::template run<T, 3, false, true, true>(v, lds, m, r, rw, p, d, tw);
    __syncthreads();                                       // the last stage read LDS
    F::template run<T, 3, false, true, true>(v + 3, lds, m, r, rw, p, d, tw);
  }
  if (a.mode & (XM_PROJ | XM_DIV | XM_DISP)) {
    const double sy = sym[nx + ky], sz = sym[nx + a.ny + kz];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int kx = p + i * P;
      C A[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) A[c] = v[c][i];
      if (a.mode & XM_PROJ) project_one<T>(A, sym[kx], sy, sz);
      else vector_op<T>(a.mode, A, sym[kx], sy, sz, a.h);
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c][i] = A[c];
    }
  }
  if (a.mode & XM_INV) {
    if (a.mode & XM_FWD) __syncthreads();                  // forward's last stage read LDS
    F::template run<T, 3, true, true, true>(v, lds, m, r, rw, p, d, tw);
    __syncthreads();
    F::template run<T, 3, true, true, true>(v + 3, lds, m, r, rw, p, d, tw);
  }
  const int ncomp_out = (a.mode & (XM_DIV | XM_DISP)) ? 3 : 6;
  if (valid) {
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (c < ncomp_out)
#pragma unroll
        for (int i = 0; i < E; ++i) W[base + c * cstride + (size_t)i * P] = v[c][i];
  }
}

// Swap between the two halves of a wavefront (v_permlane32_swap exchanges lanes 32..63
// of its first operand with lanes 0..31 of its second).  Afterwards, in lane l < 32, lo
// is unchanged and hi holds the lo of lane l + 32; in lane l >= 32, lo holds the hi of
// lane l - 32 and hi is unchanged.
__device__ __forceinline__ void half_swap_w(float& lo, float& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
  lo = __uint_as_float(r[0]);
  hi = __uint_as_float(r[1]);
}
__device__ __forceinline__ void half_swap_w(double& lo, double& hi) {
  unsigned long long a = __double_as_longlong(lo), b = __double_as_longlong(hi);
  const auto r0 = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
  const auto r1 = __builtin_amdgcn_permlane32_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
  lo = __longlong_as_double((long long)(((unsigned long long)r1[0] << 32) | r0[0]));
  hi = __longlong_as_double((long long)(((unsigned long long)r1[1] << 32) | r0[1]));
}
template <typename T>
__device__ __forceinline__ void half_swap(cplx<T>& lo, cplx<T>& hi) {
  half_swap_w(lo.x, hi.x);
  half_swap_w(lo.y, hi.y);
}

// Six-component x pass split over the halves of a wavefront: lanes 0..31 hold the three
// normal components (slots 0..2) and lanes 32..63 the three shear components (slots
// 3..5) of the same rows, E elements p + i*P each, so a lane carries half the registers
// of k_x6_r and transforms three rows.  For the per-frequency operation the halves
// divide the frequencies: lanes 0..31 take elements i < E/2, lanes 32..63 elements
// i >= E/2.  One swap per value brings the six components of a lane's frequency
// together, a second returns the results to the lanes that own them.  P = nx / E
// divides 32, so 32 / P rows share a wavefront.
template <typename T, typename F>
__global__ __launch_bounds__(kMaxFastThreads) void k_x6s_r(cplx<T>* __restrict__ W, XArgs a, FftDesc d,
                                                           const cplx<T>* __restrict__ tw,
                                                           const double* __restrict__ sym) {
  using C = cplx<T>;
  constexpr int E = F::E, EH = E / 2;
  static_assert(E % 2 == 0, "the halves split the elements of a lane in two");
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int nx = F::len(d), P = nx / E;
  const int lane = threadIdx.x & 63, half = lane >> 5, sub = lane & 31;
  const int p = sub % P;
  const int rl = (threadIdx.x >> 6) * (32 / P) + sub / P;   // row of the workgroup
  const int row = blockIdx.x * a.rw + rl;
  const bool valid = rl < a.rw && row < a.rows;
  const size_t cstride = (size_t)a.nzh * a.ny * nx;
  int kz = 0, ky = 0;
  const size_t base = valid ? x_row_base(a, row, 0, kz, ky) + (size_t)(3 * half) * cstride + p : 0;
  C v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < E; ++i) v[c][i] = valid ? W[base + c * cstride + (size_t)i * P] : mk<T>((T)0, (T)0);
  const LdsMap m{nx + (nx >> kX6Skew) + 1, 1, kX6Skew};
  const int line0 = (rl * 2 + half) * 3;
  if (a.mode & XM_FWD) F::template run<T, 3, false, true, true>(v, lds, m, line0, 1, p, d, tw);
  if (a.mode & (XM_PROJ | XM_DIV | XM_DISP)) {
    const double sy = sym[nx + ky], sz = sym[nx + a.ny + kz];
#pragma unroll
    for (int j = 0; j < EH; ++j) {
      C A[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        A[c] = v[c][j];
        A[3 + c] = v[c][j + EH];
        half_swap<T>(A[c], A[3 + c]);        // the six components of element j + half * EH
      }
      const double sx = sym[p + (j + half * EH) * P];
      if (a.mode & XM_PROJ) project_one<T>(A, sx, sy, sz);
      else vector_op<T>(a.mode, A, sx, sy, sz, a.h);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        half_swap<T>(A[c], A[3 + c]);        // back: component c (lo) or 3 + c (hi) of j and j + EH
        v[c][j] = A[c];
        v[c][j + EH] = A[3 + c];
      }
    }
  }
  if (a.mode & XM_INV) {
    if (a.mode & XM_FWD) __syncthreads();                  // forward's last stage read LDS
    F::template run<T, 3, true, true, true>(v, lds, m, line0, 1, p, d, tw);
  }
  const bool store = valid && (half == 0 || !(a.mode & (XM_DIV | XM_DISP)));
  if (store) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < E; ++i) W[base + c * cstride + (size_t)i * P] = v[c][i];
  }
}

// Select between two complex values by value (a conditional on array elements would
// select their addresses and keep the arrays out of registers).
template <typename T>
__device__ __forceinline__ cplx<T> csel(bool s, cplx<T> a, cplx<T> b) {
  return mk<T>(s ? a.x : b.x, s ? a.y : b.y);
}

// The same split for lines of 64 threads (P = nx / E = 64, e.g. 512 = 64 x 8): the three
// normal components of a row sit in one wavefront and the three shear components in the
// next, so the per-frequency exchange goes through LDS instead of a lane swap.  Wavefront
// h of row r takes frequencies i in [h E/2, (h + 1) E/2): it writes its components of the
// other half to LDS, reads the other wavefront's components of its own half, evaluates
// the operation, keeps its own components and writes the other wavefront's back.  The
// exchange reuses the row's six FFT lines (3 * E * 64 values fit in them).
template <typename T, typename F>
__global__ __launch_bounds__(kMaxFastThreads) void k_x6w_r(cplx<T>* __restrict__ W, XArgs a, FftDesc d,
                                                           const cplx<T>* __restrict__ tw,
                                                           const double* __restrict__ sym) {
  using C = cplx<T>;
  constexpr int E = F::E, EH = E / 2, P = 64;
  static_assert(E % 2 == 0 && F::N / F::E == 64, "one wavefront per component triple of a line");
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int nx = F::len(d);
  const int p = threadIdx.x & 63, w = threadIdx.x >> 6, h = w & 1, rl = w >> 1;
  const int row = blockIdx.x * a.rw + rl;
  const bool valid = rl < a.rw && row < a.rows;
  const size_t cstride = (size_t)a.nzh * a.ny * nx;
  int kz = 0, ky = 0;
  const size_t base = valid ? x_row_base(a, row, 0, kz, ky) + (size_t)(3 * h) * cstride + p : 0;
  C v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < E; ++i) v[c][i] = valid ? W[base + c * cstride + (size_t)i * P] : mk<T>((T)0, (T)0);
  const LdsMap m{nx + (nx >> kX6Skew) + 1, 1, kX6Skew};
  const int line0 = (rl * 2 + h) * 3;
  if (a.mode & XM_FWD) F::template run<T, 3, false, true, true>(v, lds, m, line0, 1, p, d, tw);
  if (a.mode & (XM_PROJ | XM_DIV | XM_DISP)) {
    // per row: X_h, then Y_h, each 3 * EH * 64 values, in the row's own six lines
    C* rowl = lds + (size_t)rl * 6 * m.ls;
    C* X = rowl;
    C* Y = rowl + 2 * 3 * EH * P;
    auto at = [&](int hh, int c, int j) { return (hh * 3 * EH + c * EH + j) * P + p; };
    __syncthreads();                                        // the forward's last stage read LDS
    // (register indices stay compile-time: the wavefront's half picks values by select)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < EH; ++j) X[at(h, c, j)] = csel<T>(h, v[c][j], v[c][j + EH]);
    __syncthreads();
    const double sy = sym[nx + ky], sz = sym[nx + a.ny + kz];
#pragma unroll
    for (int j = 0; j < EH; ++j) {
      C A[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const C other = X[at(1 - h, c, j)];
        const C own = csel<T>(h, v[c][j + EH], v[c][j]);
        A[c] = csel<T>(h, other, own);
        A[3 + c] = csel<T>(h, own, other);
      }
      const double sx = sym[p + (j + h * EH) * P];
      if (a.mode & XM_PROJ) project_one<T>(A, sx, sy, sz);
      else vector_op<T>(a.mode, A, sx, sy, sz, a.h);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[c][j + EH] = csel<T>(h, A[3 + c], v[c][j + EH]);
        v[c][j] = csel<T>(h, v[c][j], A[c]);
        Y[at(h, c, j)] = csel<T>(h, A[c], A[3 + c]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < EH; ++j) {
        const C back = Y[at(1 - h, c, j)];
        v[c][j] = csel<T>(h, back, v[c][j]);
        v[c][j + EH] = csel<T>(h, v[c][j + EH], back);
      }
    __syncthreads();                                        // the inverse writes these lines
  }
  if (a.mode & XM_INV) {
    if ((a.mode & XM_FWD) && !(a.mode & (XM_PROJ | XM_DIV | XM_DISP))) __syncthreads();
    F::template run<T, 3, true, true, true>(v, lds, m, line0, 1, p, d, tw);
  }
  const bool store = valid && (h == 0 || !(a.mode & (XM_DIV | XM_DISP)));
  if (store) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < E; ++i) W[base + c * cstride + (size_t)i * P] = v[c][i];
  }
}

// ------------------------------------------------------- launch helper -----

enum KernelKind : int { KK_Z_R2C, KK_Z_C2R, KK_Y_FWD, KK_Y_INV, KK_X, KK_X6, KK_X6S };

// Everything one register-engine launch needs; launch_with<T, F> issues it.
template <typename T>
struct FastArgs {
  KernelKind kind;
  int n, E;                     // line length and elements per thread of the pass's axis
  bool dry = false;             // only report whether a compile-time schedule serves the launch
  dim3 grid, block;
  size_t lds;
  hipStream_t s;
  FftDesc d;
  const cplx<T>* tw;
  // z_r2c
  const T* in = nullptr;
  cplx<T>* W = nullptr;
  ZArgs za{};
  // z_c2r
  const cplx<T>* Wc = nullptr;
  T* out = nullptr;
  T* removed = nullptr;
  ZcArgs zca{};
  T scale = (T)1;
  // y / x
  YArgs ya{};
  XArgs xa{};
  const double* sym = nullptr;
};

template <typename T, typename F>
void launch_with(const FastArgs<T>& a) {
  switch (a.kind) {
    case KK_Z_R2C:
      hipLaunchKernelGGL((k_z_r2c_r<T, F>), a.grid, a.block, a.lds, a.s, a.in, a.W, a.za, a.d, a.tw);
      break;
    case KK_Z_C2R:
      hipLaunchKernelGGL((k_z_c2r_r<T, F>), a.grid, a.block, a.lds, a.s, a.Wc, a.out, a.in, a.removed, a.zca, a.d,
                         a.tw, a.scale);
      break;
    case KK_Y_FWD:
      hipLaunchKernelGGL((k_y_r<T, F, false>), a.grid, a.block, a.lds, a.s, a.W, a.ya, a.d, a.tw);
      break;
    case KK_Y_INV:
      hipLaunchKernelGGL((k_y_r<T, F, true>), a.grid, a.block, a.lds, a.s, a.W, a.ya, a.d, a.tw);
      break;
    case KK_X:
      hipLaunchKernelGGL((k_x_r<T, F>), a.grid, a.block, a.lds, a.s, a.W, a.xa, a.d, a.tw, a.sym);
      break;
    case KK_X6S:
      if constexpr (F::ct) {
        if constexpr (F::E % 2 == 0 && F::N / F::E <= 32)
          hipLaunchKernelGGL((k_x6s_r<T, F>), a.grid, a.block, a.lds, a.s, a.W, a.xa, a.d, a.tw, a.sym);
        else if constexpr (F::E % 2 == 0 && F::N / F::E == 64)
          hipLaunchKernelGGL((k_x6w_r<T, F>), a.grid, a.block, a.lds, a.s, a.W, a.xa, a.d, a.tw, a.sym);
      }
      break;
    default:
      if constexpr (F::E == 8)
        hipLaunchKernelGGL((k_x6_r<T, F>), a.grid, a.block, a.lds, a.s, a.W, a.xa, a.d, a.tw, a.sym);
      break;
  }
}

// Compile-time schedule launchers (eq_sched_*.hip); each returns false when it has no
// schedule for (n, E).
template <typename T> bool ct_launch_pow2(const FastArgs<T>& a);
template <typename T> bool ct_launch_mixed(const FastArgs<T>& a);

}  // namespace eq
