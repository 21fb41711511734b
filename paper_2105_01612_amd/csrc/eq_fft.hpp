// eq_fft.hpp -- mixed-radix FFT engine for gfx950 (device) with a host build of
// the same arithmetic for emulation on the CPU.
//
// Two engines transform lines of length n (unnormalized; forward uses
// exp(-2 pi i jk/n), inverse exp(+2 pi i jk/n)):
//
// * Register engine (line_fft): the P = n/E threads of a line each own the E
//   elements p + i*P (i < E).  Every Stockham autosort stage of radix R (R | E)
//   gives a thread the E/R butterflies j = p + m*P; their inputs j + r*n/R are
//   exactly elements p + (m + r*E/R)*P, and the outputs of the final stage land
//   on the same elements.  So the first stage can consume registers loaded
//   straight from global memory and the last stage can leave its outputs in
//   registers for a direct store; intermediate stages exchange through LDS.
// * Generic engine (fft_lines): any radix schedule, every stage staged through
//   LDS, butterflies distributed with guards.  Used for sizes the register
//   engine does not schedule (e.g. edges with both 3 and 5 as factors).
//
// Stage twiddles come from a table tw[m] = exp(-2 pi i m / n) generated in FP64
// on the device (rounded once for FP32).
#pragma once

#include <hip/hip_runtime.h>

#define EQ_HD __host__ __device__ __forceinline__

namespace eq {

template <typename T> struct cvec;
template <> struct cvec<float>  { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename T> EQ_HD cplx<T> mk(T re, T im) { cplx<T> c; c.x = re; c.y = im; return c; }
template <typename C> EQ_HD C cadd(C a, C b) { C c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }
template <typename C> EQ_HD C csub(C a, C b) { C c; c.x = a.x - b.x; c.y = a.y - b.y; return c; }
template <typename C> EQ_HD C cmul(C a, C b) {
  C c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c;
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> EQ_HD C mul_mi(C a) {
  C c;
  if (INV) { c.x = -a.y; c.y = a.x; } else { c.x = a.y; c.y = -a.x; }
  return c;
}
// multiply by exp(-i theta) (forward) or exp(+i theta) (inverse), given cos and sin of theta
template <bool INV, typename C, typename S> EQ_HD C rot(C a, S cs, S sn) {
  C c;
  if (INV) { c.x = a.x * cs - a.y * sn; c.y = a.x * sn + a.y * cs; }
  else     { c.x = a.x * cs + a.y * sn; c.y = a.y * cs - a.x * sn; }
  return c;
}
template <typename C, typename S> EQ_HD C cscale(C a, S s) { C c; c.x = a.x * s; c.y = a.y * s; return c; }

constexpr int kMaxStages = 12;
struct FftDesc {
  int n;                 // line length
  int nst;               // number of stages
  int r[kMaxStages];     // radices, product == n
};

// ------------------------------------------------------------ butterflies --

template <int R, bool INV, typename C> struct Dft;

template <bool INV, typename C> struct Dft<2, INV, C> {
  static EQ_HD void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  }
};

template <bool INV, typename C> struct Dft<4, INV, C> {
  static EQ_HD void run(C* v) {
    C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2); v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3); v[3] = csub(t1, t3);
  }
};

template <bool INV, typename C> struct Dft<8, INV, C> {
  static EQ_HD void run(C* v) {
    using T = decltype(v[0].x);
    const T h = (T)0.70710678118654752440084436210484903928;   // sqrt(1/2)
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV, C>::run(e);
    Dft<4, INV, C>::run(o);
    const C o1 = rot<INV>(o[1], h, h);          // w8^1
    const C o2 = mul_mi<INV>(o[2]);             // w8^2
    const C o3 = rot<INV>(o[3], -h, h);         // w8^3
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
  }
};

// 16 = 4 x 4: inner DFT4 over n1 (stride 4), twiddle w16^(n2 k1), outer DFT4 over n2.
template <bool INV, typename C> struct Dft<16, INV, C> {
  static EQ_HD void run(C* v) {
    using T = decltype(v[0].x);
    const T c1 = (T)0.92387953251128675612818318939678828682;   // cos(pi/8)
    const T s1 = (T)0.38268343236508977172845998403039886676;   // sin(pi/8)
    const T h = (T)0.70710678118654752440084436210484903928;
    C y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      C a[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
      Dft<4, INV, C>::run(a);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = a[k1];
    }
    // twiddles w16^(n2*k1), n2, k1 in 1..3: exponents 1,2,3,2,4,6,3,6,9
    y[1][1] = rot<INV>(y[1][1], c1, s1);
    y[1][2] = rot<INV>(y[1][2], h, h);
    y[1][3] = rot<INV>(y[1][3], s1, c1);
    y[2][1] = rot<INV>(y[2][1], h, h);
    y[2][2] = mul_mi<INV>(y[2][2]);
    y[2][3] = rot<INV>(y[2][3], -h, h);
    y[3][1] = rot<INV>(y[3][1], s1, c1);
    y[3][2] = rot<INV>(y[3][2], -h, h);
    y[3][3] = rot<INV>(y[3][3], -c1, -s1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C b[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<4, INV, C>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
  }
};

template <bool INV, typename C> struct Dft<3, INV, C> {
  static EQ_HD void run(C* v) {
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
  static EQ_HD void run(C* v) {
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

// ------------------------------------------------------- register engine --

// LDS placement of element idx of a line: line * ls + idx * es (+ idx >> skew, which breaks
// the power-of-two strides of Stockham writes on contiguous lines).  kSkew is the usual shift.
constexpr int kSkew = 4;
struct LdsMap {
  int ls, es, skew;   // skew: one pad element every 2^skew elements (0: none)
  EQ_HD int at(int line, int idx) const { return line * ls + idx * es + (skew ? (idx >> skew) : 0); }
};

// j mod Ns; Ns is a power of two except after a radix-3/5 stage (those come last in a schedule).
EQ_HD int mod_ns(int j, int Ns) { return (Ns & (Ns - 1)) == 0 ? (j & (Ns - 1)) : (j % Ns); }

// Stage modes: where the inputs come from and where the outputs go.
enum StageMode : int { SM_RR = 0, SM_RL = 1, SM_LR = 2, SM_LL = 3 };

// Part A of one stage for one thread: gather, twiddle and DFT its E/R butterflies.
// RR/LR modes leave outputs in v (final placement), RL writes them to LDS at once,
// LL leaves them in v in butterfly order for part B (after a barrier).
template <typename T, int E, int R, bool INV, int MODE>
EQ_HD void stage_a(cplx<T>* v, cplx<T>* lds, const LdsMap& m, int line, int p, int n, int Ns,
                   const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int MB = E / R;
  const int P = n / E;
  const int nb = n / R;
  const int tws = n / (Ns * R);
  constexpr bool from_regs = (MODE == SM_RR || MODE == SM_RL);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int j = p + mb * P;
    const int k = mod_ns(j, Ns);
    C x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = from_regs ? v[mb + r * MB] : lds[m.at(line, j + r * nb)];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tw[r * k * tws];
        if (INV) w.y = -w.y;
        x[r] = cmul(x[r], w);
      }
    }
    Dft<R, INV, C>::run(x);
    // Outputs go straight to their destination: butterfly mb reads and writes only its
    // own register slots mb + r*MB (RR), and reads LDS when it writes registers (LR, LL).
    const int o = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (MODE == SM_RR || MODE == SM_LR) v[mb + r * MB] = x[r];      // last stage: o + r*Ns = p + (mb + r*MB)*P
      else if (MODE == SM_RL) lds[m.at(line, o + r * Ns)] = x[r];
      else v[mb * R + r] = x[r];
    }
  }
}

// Part B of an LDS-to-LDS stage: scatter the results held in v.
template <typename T, int E, int R>
EQ_HD void stage_b(const cplx<T>* v, cplx<T>* lds, const LdsMap& m, int line, int p, int n, int Ns) {
  constexpr int MB = E / R;
  const int P = n / E;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int j = p + mb * P;
    const int k = mod_ns(j, Ns);
    const int o = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) lds[m.at(line, o + r * Ns)] = v[mb * R + r];
  }
}

template <int E, int R> struct RadixOk { static constexpr bool value = (E % R) == 0; };

// Mode of stage s of nst given where the line starts (IN_REGS) and must end (OUT_REGS).
EQ_HD int stage_mode(int s, int nst, bool in_regs, bool out_regs) {
  const bool fr = (s == 0) && in_regs;
  const bool tr = (s == nst - 1) && out_regs;
  return fr ? (tr ? SM_RR : SM_RL) : (tr ? SM_LR : SM_LL);
}

#ifdef __HIP_DEVICE_COMPILE__
#define EQ_SYNC() __syncthreads()
#else
#define EQ_SYNC() ((void)0)
#endif

template <typename T, int E, int R, bool INV>
__device__ __forceinline__ void run_stage(cplx<T>* v, cplx<T>* lds, const LdsMap& m, int line, int p, int n, int Ns,
                                          const cplx<T>* __restrict__ tw, int mode, bool active) {
  if constexpr (RadixOk<E, R>::value) {
    switch (mode) {
      case SM_RR:
        if (active) stage_a<T, E, R, INV, SM_RR>(v, lds, m, line, p, n, Ns, tw);
        break;
      case SM_RL:
        if (active) stage_a<T, E, R, INV, SM_RL>(v, lds, m, line, p, n, Ns, tw);
        EQ_SYNC();
        break;
      case SM_LR:
        if (active) stage_a<T, E, R, INV, SM_LR>(v, lds, m, line, p, n, Ns, tw);
        break;
      default:
        if (active) stage_a<T, E, R, INV, SM_LL>(v, lds, m, line, p, n, Ns, tw);
        EQ_SYNC();
        if (active) stage_b<T, E, R>(v, lds, m, line, p, n, Ns);
        EQ_SYNC();
        break;
    }
  }
}

// Transform one line per thread group.  IN_REGS: v holds the input elements p + i*P
// (else the line is in LDS and visible); OUT_REGS: on return v holds the output
// elements p + i*P (else the output is in LDS, natural order, after a barrier).
// The caller guarantees no thread still reads LDS when a stage starts writing it:
// with IN_REGS the first stage writes LDS without a barrier.  Every thread of the
// block must call this (barriers); inactive threads pass active = false.
template <typename T, int E, bool INV, bool IN_REGS, bool OUT_REGS>
__device__ __forceinline__ void line_fft(cplx<T>* v, cplx<T>* lds, const LdsMap& m, int line, int p, const FftDesc& d,
                                         const cplx<T>* __restrict__ tw, bool active) {
  int Ns = 1;
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.r[s];
    const int mode = stage_mode(s, d.nst, IN_REGS, OUT_REGS);
    switch (R) {
      case 16: run_stage<T, E, 16, INV>(v, lds, m, line, p, d.n, Ns, tw, mode, active); break;
      case 8: run_stage<T, E, 8, INV>(v, lds, m, line, p, d.n, Ns, tw, mode, active); break;
      case 4: run_stage<T, E, 4, INV>(v, lds, m, line, p, d.n, Ns, tw, mode, active); break;
      case 2: run_stage<T, E, 2, INV>(v, lds, m, line, p, d.n, Ns, tw, mode, active); break;
      case 3: run_stage<T, E, 3, INV>(v, lds, m, line, p, d.n, Ns, tw, mode, active); break;
      default: run_stage<T, E, 5, INV>(v, lds, m, line, p, d.n, Ns, tw, mode, active); break;
    }
    Ns *= R;
  }
}

// NL lines per thread (lines line0 + l * lstride, l < NL), sharing every barrier.
template <typename T, int E, int R, bool INV, int NL>
__device__ __forceinline__ void run_stage_multi(cplx<T> (*v)[E], cplx<T>* lds, const LdsMap& m, int line0,
                                                int lstride, int p, int n, int Ns, const cplx<T>* __restrict__ tw,
                                                int mode) {
  if constexpr (RadixOk<E, R>::value) {
    switch (mode) {
      case SM_RR:
#pragma unroll
        for (int l = 0; l < NL; ++l) stage_a<T, E, R, INV, SM_RR>(v[l], lds, m, line0 + l * lstride, p, n, Ns, tw);
        break;
      case SM_RL:
#pragma unroll
        for (int l = 0; l < NL; ++l) stage_a<T, E, R, INV, SM_RL>(v[l], lds, m, line0 + l * lstride, p, n, Ns, tw);
        EQ_SYNC();
        break;
      case SM_LR:
#pragma unroll
        for (int l = 0; l < NL; ++l) stage_a<T, E, R, INV, SM_LR>(v[l], lds, m, line0 + l * lstride, p, n, Ns, tw);
        break;
      default:
#pragma unroll
        for (int l = 0; l < NL; ++l) stage_a<T, E, R, INV, SM_LL>(v[l], lds, m, line0 + l * lstride, p, n, Ns, tw);
        EQ_SYNC();
#pragma unroll
        for (int l = 0; l < NL; ++l) stage_b<T, E, R>(v[l], lds, m, line0 + l * lstride, p, n, Ns);
        EQ_SYNC();
        break;
    }
  }
}

// Multi-line variant of line_fft: one thread owns the same element positions of NL
// lines, so per-element work across the lines (e.g. a 6-component projection) can
// run in registers between a forward and an inverse transform.  Same LDS contract
// as line_fft; with OUT_REGS the last stage reads LDS, so a caller that writes LDS
// next must take a barrier first.
template <typename T, int E, int NL, bool INV, bool IN_REGS, bool OUT_REGS>
__device__ __forceinline__ void line_fft_multi(cplx<T> (*v)[E], cplx<T>* lds, const LdsMap& m, int line0,
                                               int lstride, int p, const FftDesc& d,
                                               const cplx<T>* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.r[s];
    const int mode = stage_mode(s, d.nst, IN_REGS, OUT_REGS);
    switch (R) {
      case 16: run_stage_multi<T, E, 16, INV, NL>(v, lds, m, line0, lstride, p, d.n, Ns, tw, mode); break;
      case 8: run_stage_multi<T, E, 8, INV, NL>(v, lds, m, line0, lstride, p, d.n, Ns, tw, mode); break;
      case 4: run_stage_multi<T, E, 4, INV, NL>(v, lds, m, line0, lstride, p, d.n, Ns, tw, mode); break;
      case 2: run_stage_multi<T, E, 2, INV, NL>(v, lds, m, line0, lstride, p, d.n, Ns, tw, mode); break;
      case 3: run_stage_multi<T, E, 3, INV, NL>(v, lds, m, line0, lstride, p, d.n, Ns, tw, mode); break;
      default: run_stage_multi<T, E, 5, INV, NL>(v, lds, m, line0, lstride, p, d.n, Ns, tw, mode); break;
    }
    Ns *= R;
  }
}

// Compile-time schedule: radices Rs..., line length N, stages S = 0.. with Ns = product
// of the radices before S.  The stage helpers see constant n and Ns, so index
// arithmetic folds and only the live stage code is emitted.
template <typename T, int E, int NL, bool INV, bool IN_REGS, bool OUT_REGS, int N, int Ns, int S, int NST, int R,
          int... Rest>
__device__ __forceinline__ void ct_multi(cplx<T> (*v)[E], cplx<T>* lds, const LdsMap& m, int line0, int lstride,
                                         int p, const cplx<T>* __restrict__ tw) {
  static_assert(E % R == 0, "radix must divide E");
  constexpr bool fr = (S == 0) && IN_REGS;
  constexpr bool tr = (S == NST - 1) && OUT_REGS;
  if constexpr (fr && tr) {
#pragma unroll
    for (int l = 0; l < NL; ++l) stage_a<T, E, R, INV, SM_RR>(v[l], lds, m, line0 + l * lstride, p, N, Ns, tw);
  } else if constexpr (fr) {
#pragma unroll
    for (int l = 0; l < NL; ++l) stage_a<T, E, R, INV, SM_RL>(v[l], lds, m, line0 + l * lstride, p, N, Ns, tw);
    EQ_SYNC();
  } else if constexpr (tr) {
#pragma unroll
    for (int l = 0; l < NL; ++l) stage_a<T, E, R, INV, SM_LR>(v[l], lds, m, line0 + l * lstride, p, N, Ns, tw);
  } else {
#pragma unroll
    for (int l = 0; l < NL; ++l) stage_a<T, E, R, INV, SM_LL>(v[l], lds, m, line0 + l * lstride, p, N, Ns, tw);
    EQ_SYNC();
#pragma unroll
    for (int l = 0; l < NL; ++l) stage_b<T, E, R>(v[l], lds, m, line0 + l * lstride, p, N, Ns);
    EQ_SYNC();
  }
  if constexpr (sizeof...(Rest) > 0)
    ct_multi<T, E, NL, INV, IN_REGS, OUT_REGS, N, Ns * R, S + 1, NST, Rest...>(v, lds, m, line0, lstride, p, tw);
}

constexpr int gcd_ct(int a, int b) { return b == 0 ? a : gcd_ct(b, a % b); }
constexpr int lcm_ct(int a, int b) { return a / gcd_ct(a, b) * b; }
template <int... Rs> struct LcmOf;
template <int R> struct LcmOf<R> { static constexpr int value = R; };
template <int R, int... Rest> struct LcmOf<R, Rest...> {
  static constexpr int value = lcm_ct(R, LcmOf<Rest...>::value);
};

// FFT policies used by the kernels.  Both expose E (elements per thread), len(d) (the
// line length: a constant for a compile-time schedule) and run<T, NL, INV, IN, OUT>().
// Sched<R...>: compile-time radix schedule (index arithmetic folds, only live stage
// code is emitted); RtFft<E>: radices read from the FftDesc at run time.
template <int... Rs> struct Sched {
  static constexpr bool ct = true;
  static constexpr int N = (Rs * ...);
  static constexpr int nst = sizeof...(Rs);
  static constexpr int E = LcmOf<Rs...>::value;
  static EQ_HD constexpr int len(const FftDesc&) { return N; }
  template <typename T, int NL, bool INV, bool IN_REGS, bool OUT_REGS>
  static __device__ __forceinline__ void run(cplx<T> (*v)[E], cplx<T>* lds, const LdsMap& m, int line0, int lstride,
                                             int p, const FftDesc&, const cplx<T>* __restrict__ tw) {
    ct_multi<T, E, NL, INV, IN_REGS, OUT_REGS, N, 1, 0, nst, Rs...>(v, lds, m, line0, lstride, p, tw);
  }
};

template <int E_> struct RtFft {
  static constexpr bool ct = false;
  static constexpr int E = E_;
  static EQ_HD int len(const FftDesc& d) { return d.n; }
  template <typename T, int NL, bool INV, bool IN_REGS, bool OUT_REGS>
  static __device__ __forceinline__ void run(cplx<T> (*v)[E], cplx<T>* lds, const LdsMap& m, int line0, int lstride,
                                             int p, const FftDesc& d, const cplx<T>* __restrict__ tw) {
    line_fft_multi<T, E, NL, INV, IN_REGS, OUT_REGS>(v, lds, m, line0, lstride, p, d, tw);
  }
};

// ------------------------------------------------------- generic engine ---

// One Stockham stage of radix R on all lines held in LDS, butterflies spread over
// P = n / E threads per line with guards (R need not divide E).
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

// Transform all lines in LDS.  Threads map to (line, p) with line fastest; thread
// tid >= nlines * (n / E) idles but still takes every barrier.
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
