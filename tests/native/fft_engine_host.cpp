// Host emulation of the register FFT engine (eq_fft.hpp): every thread of one
// line runs stage part A, then (LDS-to-LDS stages) part B, in the same order the
// device barriers impose; the result is compared with a direct O(n^2) DFT.
// Prints one line per case: "<n> <E> <dir> <prec> <rel_err>".
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "eq_fft.hpp"

using namespace eq;

template <typename T, int E, bool INV>
double run_case(const FftDesc& d, bool in_regs, bool out_regs, unsigned seed) {
  using C = cplx<T>;
  const int n = d.n, P = n / E;
  std::vector<C> tw(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    tw[m] = mk<T>((T)std::cos(a), (T)std::sin(a));
  }
  std::vector<std::complex<double>> x(n);
  srand(seed);
  for (int i = 0; i < n; ++i) x[i] = {rand() / (double)RAND_MAX - 0.5, rand() / (double)RAND_MAX - 0.5};
  // one line, skewed contiguous layout
  LdsMap m{n + (n >> kSkew) + 1, 1, kSkew};
  std::vector<C> lds(m.ls);
  std::vector<std::vector<C>> v(P, std::vector<C>(E));
  for (int p = 0; p < P; ++p)
    for (int i = 0; i < E; ++i) {
      const int idx = p + i * P;
      const C c = mk<T>((T)x[idx].real(), (T)x[idx].imag());
      if (in_regs) v[p][i] = c; else lds[m.at(0, idx)] = c;
    }
  int Ns = 1;
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.r[s];
    const int mode = stage_mode(s, d.nst, in_regs, out_regs);
    for (int p = 0; p < P; ++p) {
      C* vp = v[p].data();
#define EQ_A(RR)                                                                                              \
  if constexpr (E % RR == 0) {                                                                                 \
    if (mode == SM_RR) stage_a<T, E, RR, INV, SM_RR>(vp, lds.data(), m, 0, p, n, Ns, tw.data());               \
    else if (mode == SM_RL) stage_a<T, E, RR, INV, SM_RL>(vp, lds.data(), m, 0, p, n, Ns, tw.data());          \
    else if (mode == SM_LR) stage_a<T, E, RR, INV, SM_LR>(vp, lds.data(), m, 0, p, n, Ns, tw.data());          \
    else stage_a<T, E, RR, INV, SM_LL>(vp, lds.data(), m, 0, p, n, Ns, tw.data());                            \
  } else { std::printf("bad radix\n"); std::exit(2); }
      switch (R) {
        case 16: EQ_A(16) break;
        case 8: EQ_A(8) break;
        case 4: EQ_A(4) break;
        case 2: EQ_A(2) break;
        case 3: EQ_A(3) break;
        default: EQ_A(5) break;
      }
#undef EQ_A
    }
    if (mode == SM_LL) {
      for (int p = 0; p < P; ++p) {
        C* vp = v[p].data();
        switch (R) {
          case 16: if constexpr (E % 16 == 0) stage_b<T, E, 16>(vp, lds.data(), m, 0, p, n, Ns); break;
          case 8: if constexpr (E % 8 == 0) stage_b<T, E, 8>(vp, lds.data(), m, 0, p, n, Ns); break;
          case 4: if constexpr (E % 4 == 0) stage_b<T, E, 4>(vp, lds.data(), m, 0, p, n, Ns); break;
          case 2: stage_b<T, E, 2>(vp, lds.data(), m, 0, p, n, Ns); break;
          case 3: if constexpr (E % 3 == 0) stage_b<T, E, 3>(vp, lds.data(), m, 0, p, n, Ns); break;
          default: if constexpr (E % 5 == 0) stage_b<T, E, 5>(vp, lds.data(), m, 0, p, n, Ns); break;
        }
      }
    }
    Ns *= R;
  }
  double num = 0, den = 0;
  const double sg = INV ? 1.0 : -1.0;
  for (int k = 0; k < n; ++k) {
    std::complex<double> ref = 0;
    for (int j = 0; j < n; ++j) ref += x[j] * std::polar(1.0, sg * 2.0 * M_PI * (double)((long)j * k % n) / n);
    C g;
    if (out_regs) g = v[k % P][k / P]; else g = lds[m.at(0, k)];
    const std::complex<double> gc(g.x, g.y);
    num += std::norm(gc - ref);
    den += std::norm(ref);
  }
  return std::sqrt(num / den);
}

template <typename T, int E>
void sweep(const FftDesc& d, const char* prec) {
  for (int io = 0; io < 4; ++io) {
    const bool ir = io & 1, orr = io & 2;
    const double ef = run_case<T, E, false>(d, ir, orr, 7 + io);
    const double ei = run_case<T, E, true>(d, ir, orr, 11 + io);
    std::printf("%d %d fwd %s %d%d %.3e\n", d.n, E, prec, (int)ir, (int)orr, ef);
    std::printf("%d %d inv %s %d%d %.3e\n", d.n, E, prec, (int)ir, (int)orr, ei);
  }
}

int main(int argc, char** argv) {
  // argv: E r1 r2 ... (radices)
  if (argc < 3) return 2;
  const int E = std::atoi(argv[1]);
  FftDesc d{};
  d.n = 1;
  d.nst = argc - 2;
  for (int i = 0; i < d.nst; ++i) { d.r[i] = std::atoi(argv[2 + i]); d.n *= d.r[i]; }
  switch (E) {
    case 8: sweep<double, 8>(d, "f64"); sweep<float, 8>(d, "f32"); break;
    case 16: sweep<double, 16>(d, "f64"); sweep<float, 16>(d, "f32"); break;
    case 24: sweep<double, 24>(d, "f64"); sweep<float, 24>(d, "f32"); break;
    case 40: sweep<double, 40>(d, "f64"); sweep<float, 40>(d, "f32"); break;
    case 12: sweep<double, 12>(d, "f64"); sweep<float, 12>(d, "f32"); break;
    case 20: sweep<double, 20>(d, "f64"); sweep<float, 20>(d, "f32"); break;
    default: return 2;
  }
  return 0;
}
