// Shared device-side definitions of the gfx950 kernels: per-prime constants, the limb
// maps of batched launches and cache hints.  The modular arithmetic itself (residues
// below 2^50 as binary64, Barrett products with an exact FMA remainder) is in
// modarith.hpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.hpp"

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

