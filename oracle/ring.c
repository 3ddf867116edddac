/*
 * Oracle kernels: plain, slow, exact arithmetic in Z_q[X]/(X^N + 1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file belongs to the CPU oracle that checks the
 * GPU library; only the test-suite, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code with the GPU path.
 *
 * Every routine is the textbook definition written out with 128-bit integers:
 *   - the negacyclic product is the schoolbook sum  c_k = sum_{i+j=k} a_i b_j
 *     - sum_{i+j=k+N} a_i b_j  (the ring of the scheme, Background section on BGV),
 *   - the NTT is direct evaluation of the polynomial at the odd powers of a
 *     primitive 2N-th root of unity in bit-reversed order,
 *   - elementwise products are (a*b) mod q with a 128-bit product.
 * Parallelism is only OpenMP over independent output coefficients.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

typedef unsigned __int128 u128;

static inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a * b) % q);
}

uint64_t o_powmod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}

/* out = sum_{t < n_terms} a[t] * b[t]  in Z_q[X]/(X^N+1); a, b are [n_terms][N]. */
void o_negacyclic_dot(const uint64_t* a, const uint64_t* b, int64_t n_terms, uint64_t* out,
                      int64_t N, uint64_t q) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < N; ++k) {
    u128 pos = 0, neg = 0;
    for (int64_t t = 0; t < n_terms; ++t) {
      const uint64_t* at = a + t * N;
      const uint64_t* bt = b + t * N;
      for (int64_t i = 0; i <= k; ++i) pos += (u128)at[i] * bt[k - i];
      for (int64_t i = k + 1; i < N; ++i) neg += (u128)at[i] * bt[N + k - i];
    }
    uint64_t p = (uint64_t)(pos % q), m = (uint64_t)(neg % q);
    out[k] = p >= m ? p - m : p + q - m;
  }
}

/* Selected output coefficients only: out[s] = (a * b)[idx[s]]. */
void o_negacyclic_dot_at(const uint64_t* a, const uint64_t* b, int64_t n_terms, const int64_t* idx,
                         int64_t n_idx, uint64_t* out, int64_t N, uint64_t q) {
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < n_idx; ++s) {
    int64_t k = idx[s];
    u128 pos = 0, neg = 0;
    for (int64_t t = 0; t < n_terms; ++t) {
      const uint64_t* at = a + t * N;
      const uint64_t* bt = b + t * N;
      for (int64_t i = 0; i <= k; ++i) pos += (u128)at[i] * bt[k - i];
      for (int64_t i = k + 1; i < N; ++i) neg += (u128)at[i] * bt[N + k - i];
    }
    uint64_t p = (uint64_t)(pos % q), m = (uint64_t)(neg % q);
    out[s] = p >= m ? p - m : p + q - m;
  }
}

/* Product with a small signed polynomial (e.g. the ternary secret): exact integer sums
 * c_k = sum_j s_j a_{k-j} (with a_{k-j} -> -a_{k-j+N} when k < j), taken over the nonzero s_j. */
void o_negacyclic_mul_small(const uint64_t* a, const int64_t* s, uint64_t* out, int64_t N, uint64_t q) {
  int64_t nz = 0;
  for (int64_t j = 0; j < N; ++j) nz += s[j] != 0;
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (nz ? nz : 1));
  nz = 0;
  for (int64_t j = 0; j < N; ++j)
    if (s[j]) pos[nz++] = j;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < N; ++k) {
    u128 plus = 0, minus = 0;
    for (int64_t t = 0; t < nz; ++t) {
      const int64_t j = pos[t];
      const int64_t sv = s[j];
      const uint64_t mag = (uint64_t)(sv < 0 ? -sv : sv);
      int neg = sv < 0;
      uint64_t av;
      if (j <= k) av = a[k - j]; else { av = a[N + k - j]; neg = !neg; }
      if (neg) minus += (u128)av * mag; else plus += (u128)av * mag;
    }
    uint64_t p = (uint64_t)(plus % q), m = (uint64_t)(minus % q);
    out[k] = p >= m ? p - m : p + q - m;
  }
  free(pos);
}

/* Elementwise helpers. */
void o_mulmod_vec(const uint64_t* a, const uint64_t* b, uint64_t* out, int64_t n, uint64_t q) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = mulmod(a[i], b[i], q);
}

void o_mulmod_scalar(const uint64_t* a, uint64_t s, uint64_t* out, int64_t n, uint64_t q) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = mulmod(a[i], s, q);
}

static inline int64_t bitrev(int64_t x, int logn) {
  int64_t r = 0;
  for (int b = 0; b < logn; ++b) r |= ((x >> b) & 1) << (logn - 1 - b);
  return r;
}

/* Forward negacyclic NTT by definition: out[j] = sum_i a_i psi^{(2 brv(j) + 1) i}. */
void o_ntt_def(const uint64_t* a, uint64_t* out, int64_t N, uint64_t q, uint64_t psi) {
  int logn = 0;
  while (((int64_t)1 << logn) < N) ++logn;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j) {
    uint64_t w = o_powmod(psi, (uint64_t)(2 * bitrev(j, logn) + 1), q);
    /* Horner: a(w) */
    uint64_t acc = 0;
    for (int64_t i = N - 1; i >= 0; --i) acc = (mulmod(acc, w, q) + a[i]) % q;
    out[j] = acc;
  }
}

/* Inverse by definition: a_i = N^{-1} sum_j ahat_j psi^{-(2 brv(j) + 1) i}. */
void o_intt_def(const uint64_t* ahat, uint64_t* out, int64_t N, uint64_t q, uint64_t psi,
                uint64_t* scratch /* 2N words */) {
  int logn = 0;
  while (((int64_t)1 << logn) < N) ++logn;
  uint64_t psi_inv = o_powmod(psi, q - 2, q);
  uint64_t n_inv = o_powmod((uint64_t)N % q, q - 2, q);
  /* scratch[e] = psi^{-e} for e in [0, 2N) */
  scratch[0] = 1;
  for (int64_t e = 1; e < 2 * N; ++e) scratch[e] = mulmod(scratch[e - 1], psi_inv, q);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    u128 acc = 0;
    for (int64_t j = 0; j < N; ++j) {
      uint64_t e = ((uint64_t)(2 * bitrev(j, logn) + 1) * (uint64_t)i) % (uint64_t)(2 * N);
      acc += (u128)ahat[j] * scratch[e];
    }
    out[i] = mulmod((uint64_t)(acc % q), n_inv, q);
  }
}

/* Forward NTT by definition at selected output indices only. */
void o_ntt_def_at(const uint64_t* a, const int64_t* idx, int64_t n_idx, uint64_t* out, int64_t N, uint64_t q,
                  uint64_t psi) {
  int logn = 0;
  while (((int64_t)1 << logn) < N) ++logn;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < n_idx; ++s) {
    uint64_t w = o_powmod(psi, (uint64_t)(2 * bitrev(idx[s], logn) + 1), q);
    uint64_t acc = 0;
    for (int64_t i = N - 1; i >= 0; --i) acc = (mulmod(acc, w, q) + a[i]) % q;
    out[s] = acc;
  }
}
