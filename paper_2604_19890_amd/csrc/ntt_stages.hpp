// Radix-2 butterfly stages on 16 values held in registers (one register step of an
// NTT pass), shared by the transform kernels and usable on the host, where a test
// program checks the lazy-reduction bounds stated in ntt.hip on adversarial operands.
#pragma once
#include "modarith.hpp"

// Cooley-Tukey stages at register distances DMAX, DMAX/2, .., 1 on 16 registers
// holding global indices g0 + i * 2^gs_log.  The butterflies of group g at
// distance dd share twiddle number ((N + g0) >> log2(2 dd 2^gs_log)) + g.
template <int DMAX>
MA_FN void ct_stages(double* v, const double* __restrict__ w, int N, int g0, int gs_log,
                                          double q, double qinv) {
#pragma unroll
  for (int dd = DMAX; dd >= 1; dd >>= 1) {
    const double* wp = w + ((N + g0) >> (__builtin_ctz(2 * dd) + gs_log));
#pragma unroll
    for (int g = 0; g < 16 / (2 * dd); ++g) {
      const double wt = wp[g];
#pragma unroll
      for (int i = g * 2 * dd; i < g * 2 * dd + dd; ++i) {
        const double r = mul_lazy(v[i + dd], wt, q, qinv);
        const double a = v[i];
        v[i] = a + r;
        v[i + dd] = a - r;
      }
    }
  }
}

// The twiddles ct_stages<DMAX> reads for (g0, gs_log), in the order it uses them
// (1 + 2 + .. + 8 = 15 for DMAX = 8), and the same stages taking them from that array: a
// caller that runs the stages on several rows under one prime loads them once.
template <int DMAX>
MA_FN void ct_twiddles(double* tws, const double* __restrict__ w, int N, int g0, int gs_log) {
  int n = 0;
#pragma unroll
  for (int dd = DMAX; dd >= 1; dd >>= 1) {
    const double* wp = w + ((N + g0) >> (__builtin_ctz(2 * dd) + gs_log));
#pragma unroll
    for (int g = 0; g < 16 / (2 * dd); ++g) tws[n++] = wp[g];
  }
}

template <int DMAX>
MA_FN void ct_stages_tw(double* v, const double* tws, double q, double qinv) {
  int n = 0;
#pragma unroll
  for (int dd = DMAX; dd >= 1; dd >>= 1) {
#pragma unroll
    for (int g = 0; g < 16 / (2 * dd); ++g) {
      const double wt = tws[n++];
#pragma unroll
      for (int i = g * 2 * dd; i < g * 2 * dd + dd; ++i) {
        const double r = mul_lazy(v[i + dd], wt, q, qinv);
        const double a = v[i];
        v[i] = a + r;
        v[i + dd] = a - r;
      }
    }
  }
}

// Gentleman-Sande stages at register distances 1, 2, .., DMAX.
template <int DMAX>
MA_FN void gs_stages(double* v, const double* __restrict__ w, int N, int g0, int gs_log,
                                          double q, double qinv) {
  int stage = 0;
#pragma unroll
  for (int dd = 1; dd <= DMAX; dd <<= 1) {
    ++stage;
    const double* wp = w + ((N + g0) >> (__builtin_ctz(2 * dd) + gs_log));
#pragma unroll
    for (int g = 0; g < 16 / (2 * dd); ++g) {
      const double wt = wp[g];
#pragma unroll
      for (int i = g * 2 * dd; i < g * 2 * dd + dd; ++i) {
        const double a = v[i], b = v[i + dd];
        const double s = a + b;
        v[i] = (stage & 1) ? s : red(s, q, qinv);
        v[i + dd] = mul_lazy(a - b, wt, q, qinv);
      }
    }
  }
}
