// Host-side number theory of the library: modular arithmetic on 64-bit words,
// primality, the prime chain, NTT roots and small polynomial algebra mod p^e.
#pragma once
#include <stdint.h>

#include <vector>

namespace hnt {

typedef unsigned __int128 u128;

inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

inline uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod(r, b, m);
    b = mulmod(b, b, m);
    e >>= 1;
  }
  return r;
}

// inverse by the extended Euclidean algorithm (gcd(a, m) must be 1)
inline uint64_t invmod(uint64_t a, uint64_t m) {
  __int128 t = 0, nt = 1, r = m, nr = a % m;
  while (nr) {
    __int128 qq = r / nr, tmp;
    tmp = t - qq * nt; t = nt; nt = tmp;
    tmp = r - qq * nr; r = nr; nr = tmp;
  }
  if (t < 0) t += m;
  return (uint64_t)t;
}

// Miller-Rabin with the first twelve prime bases: deterministic below 3.3e24.
inline bool is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t b : bases) {
    if (n % b == 0) return n == b;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s; ++i) {
      x = mulmod(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

inline uint64_t gcd(uint64_t a, uint64_t b) {
  while (b) { uint64_t t = a % b; a = b; b = t; }
  return a;
}

// descending primes below 2^50, >= 2^49, congruent to 1 mod M
inline bool prime_chain(uint64_t M, int count, std::vector<uint64_t>& out) {
  out.clear();
  const uint64_t top = (uint64_t)1 << 50, bottom = (uint64_t)1 << 49;
  uint64_t x = ((top - 2) / M) * M + 1;
  while ((int)out.size() < count) {
    if (x < bottom) return false;
    if (is_prime(x)) out.push_back(x);
    x -= M;
  }
  return true;
}

// smallest of the N primitive 2N-th roots of unity mod q
inline uint64_t min_root_2n(uint64_t q, uint64_t N) {
  uint64_t e = (q - 1) / (2 * N), c = 0;
  for (uint64_t x = 2;; ++x) {
    c = powmod(x, e, q);
    if (powmod(c, N, q) == q - 1) break;
  }
  uint64_t c2 = mulmod(c, c, q), w = c, best = c;
  for (uint64_t i = 1; i < N; ++i) {
    w = mulmod(w, c2, q);
    if (w < best) best = w;
  }
  return best;
}

inline uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int b = 0; b < bits; ++b) r |= ((x >> b) & 1u) << (bits - 1 - b);
  return r;
}

inline int64_t centered(int64_t x, int64_t m) {
  x %= m;
  if (x < 0) x += m;
  return x > (m - 1) / 2 ? x - m : x;
}

}  // namespace hnt
