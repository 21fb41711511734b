// eq_fft.hpp -- device-side mixed-radix FFT engine for gfx950.
//
// A workgroup transforms `nlines` independent lines of length n that live in
// LDS at lds[line * ls + i * es].  Each line is owned by P = n / E threads
// (E = nominal elements per thread, a compile-time constant); every stage of
// radix R in {2, 3, 4, 5, 8} is a Stockham autosort step: each thread loads its
// butterflies' R inputs at stride n/R, multiplies by the stage twiddles (read
// from a table generated in FP64 on the device), runs the radix-R DFT in
// registers, waits at a barrier, then writes the R outputs at stride Ns.  All
// loads of a stage complete before any store, so the transform is in place in
// LDS.  Forward uses exp(-2 pi i jk/n), inverse exp(+2 pi i jk/n); neither
// normalizes.
#pragma once

#include <hip/hip_runtime.h>

namespace eq {

template <typename T> struct cvec;
template <> struct cvec<float>  { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename T> __device__ __forceinline__ cplx<T> mk(T re, T im) { cplx<T> c; c.x = re; c.y = im; return c; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C c; c.x = a.x - b.x; c.y = a.y - b.y; return c; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c;
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C mul_mi(C a) {
  C c;
  if (INV) { c.x = -a.y; c.y = a.x; } else { c.x = a.y; c.y = -a.x; }
  return c;
}
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { C c; c.x = a.x * s; c.y = a.y * s; return c; }

constexpr int kMaxStages = 12;
struct FftDesc {
  int n;                 // line length
  int nst;               // number of stages
  int r[kMaxStages];     // radices, product == n
};

// ------------------------------------------------------------ butterflies --

template <int R, bool INV, typename C> struct Dft;

template <bool INV, typename C> struct Dft<2, INV, C> {
  static __device__ __forceinline__ void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  }
};

template <bool INV, typename C> struct Dft<4, INV, C> {
  static __device__ __forceinline__ void run(C* v) {
    C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2); v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3); v[3] = csub(t1, t3);
  }
};

template <bool INV, typename C> struct Dft<8, INV, C> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(v[0].x);
    const T h = (T)0.70710678118654752440084436210484903928;   // sqrt(1/2)
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV, C>::run(e);
    Dft<4, INV, C>::run(o);
    // o[k] *= w8^k, w8 = exp(-+ i pi / 4)
    C o1, o3;
    if (INV) {
      o1.x = h * (o[1].x - o[1].y); o1.y = h * (o[1].x + o[1].y);
      o3.x = -h * (o[3].x + o[3].y); o3.y = h * (o[3].x - o[3].y);
    } else {
      o1.x = h * (o[1].x + o[1].y); o1.y = h * (o[1].y - o[1].x);
      o3.x = h * (o[3].y - o[3].x); o3.y = -h * (o[3].x + o[3].y);
    }
    C o2 = mul_mi<INV>(o[2]);
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
  }
};

template <bool INV, typename C> struct Dft<3, INV, C> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(v[0].x);
    const T s3 = (T)0.86602540378443864676372317075293618347;   // sin(2 pi / 3)
    C t = cadd(v[1], v[2]);
    C d = csub(v[1], v[2]);
    C m = csub(v[0], cscale(t, (T)0.5));
    C id = mul_mi<INV>(cscale(d, s3));                            // -+ i sin(2pi/3) (v1 - v2)
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, id);
    v[2] = csub(m, id);
  }
};

template <bool INV, typename C> struct Dft<5, INV, C> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(v[0].x);
    const T c1 = (T)0.30901699437494742410229341718281905886;    // cos(2 pi / 5)
    const T c2 = (T)-0.80901699437494742410229341718281905886;   // cos(4 pi / 5)
    const T s1 = (T)0.95105651629515357211643933337938214340;    // sin(2 pi / 5)
    const T s2 = (T)0.58778525229247312916870595463907276860;    // sin(4 pi / 5)
    C b1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
    C b2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
    C a0 = v[0];
    C r1 = cadd(a0, cadd(cscale(b1, c1), cscale(b2, c2)));
    C r2 = cadd(a0, cadd(cscale(b1, c2), cscale(b2, c1)));
    C i1 = mul_mi<INV>(cadd(cscale(d1, s1), cscale(d2, s2)));
    C i2 = mul_mi<INV>(csub(cscale(d1, s2), cscale(d2, s1)));
    v[0] = cadd(a0, cadd(b1, b2));
    v[1] = cadd(r1, i1); v[4] = csub(r1, i1);
    v[2] = cadd(r2, i2); v[3] = csub(r2, i2);
  }
};

// ------------------------------------------------------------------ stage --

// One Stockham stage of radix R on all lines.  tw[m] = exp(-2 pi i m / n).
template <typename T, int E, int R, bool INV>
__device__ __forceinline__ void fft_stage(cplx<T>* __restrict__ lds, int n, int Ns, int line, int p, int P,
                                          int ls, int es, const cplx<T>* __restrict__ tw, bool active) {
  using C = cplx<T>;
  constexpr int MB = (E + R - 1) / R;
  C v[MB][R];
  const int nb = n / R;
  const int tws = n / (Ns * R);
  C* base = lds + line * ls;
  if (active) {
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int j = p + m * P;
      if (j < nb) {
        const int k = j % Ns;
#pragma unroll
        for (int r = 0; r < R; ++r) v[m][r] = base[(j + r * nb) * es];
        if (Ns > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            C w = tw[r * k * tws];
            if (INV) w.y = -w.y;
            v[m][r] = cmul(v[m][r], w);
          }
        }
        Dft<R, INV, C>::run(v[m]);
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int j = p + m * P;
      if (j < nb) {
        const int k = j % Ns;
        const int o = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) base[(o + r * Ns) * es] = v[m][r];
      }
    }
  }
  __syncthreads();
}

// Transform all lines in LDS.  Threads map to (line, p) with line fastest so that
// consecutive lanes touch consecutive lines; thread tid >= nlines * (n / E) idles
// but still takes every barrier.
template <typename T, int E, bool INV>
__device__ __forceinline__ void fft_lines(cplx<T>* lds, int nlines, int ls, int es, const FftDesc& d,
                                          const cplx<T>* __restrict__ tw, int tid) {
  const int P = d.n / E;
  const int line = tid % nlines;
  const int p = tid / nlines;
  const bool active = p < P;
  int Ns = 1;
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.r[s];
    switch (R) {
      case 8: fft_stage<T, E, 8, INV>(lds, d.n, Ns, line, p, P, ls, es, tw, active); break;
      case 4: fft_stage<T, E, 4, INV>(lds, d.n, Ns, line, p, P, ls, es, tw, active); break;
      case 2: fft_stage<T, E, 2, INV>(lds, d.n, Ns, line, p, P, ls, es, tw, active); break;
      case 3: fft_stage<T, E, 3, INV>(lds, d.n, Ns, line, p, P, ls, es, tw, active); break;
      default: fft_stage<T, E, 5, INV>(lds, d.n, Ns, line, p, P, ls, es, tw, active); break;
    }
    Ns *= R;
  }
}

}  // namespace eq
