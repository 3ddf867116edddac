// Shared device-side definitions of the gfx950 kernels.
//
// Residues are stored in HBM as uint64 in [0, q) with q < 2^50.  Inside the
// kernels they are carried as IEEE binary64 values, because on CDNA4 the fp64
// FMA issues at the full VALU rate while a 64x64-bit integer product has to be
// assembled from quarter-rate 32-bit multiplies.  A modular product is a Barrett
// reduction whose quotient estimate is taken in floating point and whose
// remainder is computed exactly with FMAs:
//     h = a*b (rounded), l = fma(a, b, -h) (exact: a*b = h + l),
//     k = rint(h * (1/q)),  r = fma(-k, q, h) + l.
// For |a|, |b| <= q < 2^50 the estimate k is within 0.875 of a*b/q, so the
// exact integer r = a*b - k q satisfies |r| < q and every intermediate fits the
// 53-bit significand.  Values between stages are kept signed in (-q, q) and
// brought to [0, q) only when written back.  All kernels must be compiled with
// -ffp-contract=off so that the compiler neither fuses nor reorders these steps.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct PrimeD {
  double q;     // the prime as a double (exact)
  double qinv;  // 1/q rounded to nearest
  double ninv;  // N^-1 mod q
  double pad;
};

// Which prime each limb of a launch uses: limb l -> m = l % period;
// prime index = first + m if m < ell_q, else Lfull + (m - ell_q) (a special prime).
// If skip_alpha > 0 the launch covers ModUp output [n][dnum'][period] and skips
// the limbs of digit j (= (l / period) % dnum_p) that hold the digit's own primes.
struct LimbMap {
  int period;
  int ell_q;
  int Lfull;
  int skip_alpha;
  int dnum_p;
  int first;
  int offset;  // added to the launch's limb index before the map is applied
  // Optional physical placement: with grp > 0, launch limb l is stored at row
  // (l / grp) * grp_stride + grp_first + l % grp of the data (groups of rows at a
  // stride, e.g. the special rows of every polynomial of a wider buffer).
  int grp;
  int grp_stride;
  int grp_first;
  // Optional source placement of an out-of-place first pass (sgrp > 0): launch limb
  // l is read from row (l / sgrp) * sgrp_stride + sgrp_first + l % sgrp of the source;
  // otherwise from the row it is written to.
  int sgrp;
  int sgrp_stride;
  int sgrp_first;
};

__device__ __forceinline__ int limb_phys(const LimbMap& lm, int l) {
  return lm.grp > 0 ? (l / lm.grp) * lm.grp_stride + lm.grp_first + l % lm.grp : l;
}

__device__ __forceinline__ int limb_src(const LimbMap& lm, int l) {
  return lm.sgrp > 0 ? (l / lm.sgrp) * lm.sgrp_stride + lm.sgrp_first + l % lm.sgrp : limb_phys(lm, l);
}

__device__ __forceinline__ int limb_prime(const LimbMap& lm, int l) {
  l += lm.offset;
  int m = l % lm.period;
  return m < lm.ell_q ? lm.first + m : lm.Lfull + (m - lm.ell_q);
}

__device__ __forceinline__ bool limb_skipped(const LimbMap& lm, int l) {
  if (lm.skip_alpha <= 0) return false;
  l += lm.offset;
  int m = l % lm.period;
  int j = (l / lm.period) % lm.dnum_p;
  return m < lm.ell_q && m / lm.skip_alpha == j;
}

// A load of a word the kernel reads once and nothing reads again soon (streaming):
// the non-temporal hint keeps it from displacing data that is reused from the caches.
__device__ __forceinline__ uint64_t ld_once(const uint64_t* p) { return __builtin_nontemporal_load(p); }

// exact conversions for integers in [0, 2^52)
__device__ __forceinline__ double u2d(uint64_t x) {
  return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 4503599627370496.0;
}
__device__ __forceinline__ uint64_t d2u(double v) {
  return (uint64_t)__double_as_longlong(v + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// a*b mod q as a signed value with |r| < q; requires |a|, |b| <= q.
__device__ __forceinline__ double mul_lazy(double a, double b, double q, double qinv) {
  double h = a * b;
  double l = __builtin_fma(a, b, -h);
  double k = __builtin_rint(h * qinv);
  return __builtin_fma(-k, q, h) + l;
}

// x mod q as a signed value with |r| <= q/2 + 1; requires |x| < 2^52.
__device__ __forceinline__ double red(double x, double q, double qinv) {
  return __builtin_fma(-__builtin_rint(x * qinv), q, x);
}

// [0, q) representative of a signed value with |x| < q.
__device__ __forceinline__ double canon(double x, double q) { return x < 0.0 ? x + q : x; }

// canonical residue of a signed value with |x| < 2^52
__device__ __forceinline__ uint64_t to_u(double x, double q, double qinv) {
  return d2u(canon(red(x, q, qinv), q));
}
