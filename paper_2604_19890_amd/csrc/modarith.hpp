// Exact modular arithmetic on residues below 2^50 carried as IEEE binary64.
//
// The kernels store residues in HBM as uint64 in [0, q) with q < 2^50 and compute
// on them as doubles, because on CDNA4 the fp64 FMA issues at the full VALU rate
// while a 64x64-bit integer product has to be assembled from quarter-rate 32-bit
// multiplies.  A modular product is a Barrett reduction whose quotient estimate is
// taken in floating point and whose remainder is computed exactly with FMAs:
//     h = a*b (rounded), l = fma(a, b, -h) (exact: a*b = h + l),
//     k = rint(h * (1/q)),  r = fma(-k, q, h) + l.
// For |a| <= m q, |b| < q and q < 2^50 the estimate k is within 3 m / 8 + 1/2 of
// a*b/q (the rounding of h, of 1/q and of h/q each contribute at most 2^-53 |h/q|),
// so the exact integer r = a*b - k q satisfies |r| <= (3 m / 8 + 1/2) q, and every
// intermediate fits the 53-bit significand while m q < 2^53.  Values between steps
// are kept signed and brought to [0, q) only when written back.
//
// The functions are usable on the host as well, so that a host program can check
// these bounds on adversarial operands.  Every caller must be compiled with
// -ffp-contract=off so that the compiler neither fuses nor reorders the steps.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define MA_FN __host__ __device__ __forceinline__
#else
#define MA_FN inline
#endif

// exact conversions for integers in [0, 2^52)
MA_FN double u2d(uint64_t x) {
  return __builtin_bit_cast(double, x | 0x4330000000000000ull) - 4503599627370496.0;
}
MA_FN uint64_t d2u(double v) {
  return __builtin_bit_cast(uint64_t, v + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// a*b mod q as a signed value; |r| < q for |a|, |b| <= q (bound above for larger |a|).
MA_FN double mul_lazy(double a, double b, double q, double qinv) {
  double h = a * b;
  double l = __builtin_fma(a, b, -h);
  double k = __builtin_rint(h * qinv);
  return __builtin_fma(-k, q, h) + l;
}

// x mod q as a signed value with |r| <= q/2 + 1; requires |x| < 2^52.
MA_FN double red(double x, double q, double qinv) { return __builtin_fma(-__builtin_rint(x * qinv), q, x); }

// [0, q) representative of a signed value with |x| < q.
MA_FN double canon(double x, double q) { return x < 0.0 ? x + q : x; }

// canonical residue of a signed value with |x| < 2^52
MA_FN uint64_t to_u(double x, double q, double qinv) { return d2u(canon(red(x, q, qinv), q)); }

// Exact accumulation of small-coefficient linear combinations: a word x < 2^50 is split
// into halves xh = x >> 25 and xl = x & (2^25 - 1); with integer coefficients |c| < 2^24
// each product c xh, c xl is below 2^49 in magnitude, so the sums hi = sum c xh and
// lo = sum c xl of up to 16 terms are exact in binary64 (below 2^53).  The combination is
// then hi 2^25 + lo, reduced with one modular product.
MA_FN double split_hi(uint64_t x) { return u2d(x >> 25); }
MA_FN double split_lo(uint64_t x) { return u2d(x & 0x1FFFFFFull); }
MA_FN double split_combine(double hi, double lo, double q, double qinv) {
  return mul_lazy(red(hi, q, qinv), 33554432.0, q, qinv) + red(lo, q, qinv);
}
