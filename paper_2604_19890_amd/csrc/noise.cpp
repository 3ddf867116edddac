// Noise estimate carried with every ciphertext batch: a bound on log2 of the largest
// coefficient of [c0 + c1 s]_Q (the plaintext included), in sixteenths of a bit; 0 means
// unknown.  The paper sizes Q to the circuit's depth and leaves noise management to the
// library, so the bounds are those of the standard BGV analysis (t = p^e, n = log2 N,
// alpha = K; "6 sigma" bounds a coefficient that is a sum of many independent terms):
//   fresh encryption   |m| <= t/2, |t e| <= 19 t             -> lgc(20 t)
//   switch floor R(e)  t (tau0 + tau1 s), tau in [-1/2, 1/2]  -> lgc(3 t) - 16 + 8 n
//   modulus switch     lsum(a - Q16, R(e)), Q16 = lgf(smallest ciphertext prime)
//   tensor product     2 sqrt(N) 2^a 2^b                      -> a + b + 8 n + 16
//   key switch adds    lsum(lgc(23 alpha t) + ceil(lgc(dnum_l) / 2) + 8 n, lgc(3 alpha t) + 8 n)
//   scalar k           a + lgc(|k|);  constant k: lsum(a, lgc(|k|));  DivideByP: a - lgf(p)
//   add / sub          lsum(a, b);  tag changes, negation, dropped limbs: a
//   sum of n terms     a + lgc(n)   (each bounded by 2^a; the batch sum)
// lgc / lgf are ceil / floor of 16 log2 x, exact; lsum(a, b) bounds log2(2^a + 2^b).
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <unordered_map>

#include "ops.hpp"

namespace {

// x^16 in 32-bit words (little endian), by four exact squarings
std::vector<uint32_t> pow16(uint64_t x) {
  std::vector<uint32_t> a{(uint32_t)x, (uint32_t)(x >> 32)};
  for (int s = 0; s < 4; ++s) {
    std::vector<uint32_t> r(2 * a.size() + 1, 0);
    for (size_t i = 0; i < a.size(); ++i) {
      uint64_t carry = 0;
      for (size_t j = 0; j < a.size(); ++j) {
        const uint64_t cur = (uint64_t)a[i] * a[j] + r[i + j] + carry;
        r[i + j] = (uint32_t)cur;
        carry = cur >> 32;
      }
      for (size_t k = i + a.size(); carry; ++k) {
        const uint64_t cur = (uint64_t)r[k] + carry;
        r[k] = (uint32_t)cur;
        carry = cur >> 32;
      }
    }
    while (r.size() > 1 && r.back() == 0) r.pop_back();
    a.swap(r);
  }
  return a;
}

// floor and ceil of 16 log2 x for x >= 1: the bit length of x^16, less one unless x^16 is
// a power of two
void lg16(uint64_t x, int* fl, int* cl) {
  const std::vector<uint32_t> a = pow16(x);
  const int top = (int)a.size() - 1;
  const int bl = 32 * top + (32 - __builtin_clz(a[top]));
  bool pow2 = (a[top] & (a[top] - 1)) == 0;
  for (int i = 0; i < top && pow2; ++i) pow2 = a[i] == 0;
  *fl = bl - 1;
  *cl = pow2 ? bl - 1 : bl;
}

int lsum(int a, int b) {
  const int d = std::abs(a - b), m = std::max(a, b);
  int add;
  if (d < 16) add = 16;       // log2(1 + 2^-x) <= 1
  else if (d < 32) add = 10;  // <= log2(1.5)
  else if (d < 48) add = 6;   // <= log2(1.25)
  else if (d < 64) add = 3;   // <= log2(1.125)
  else if (d < 96) add = 2;   // <= log2(1.0625)
  else add = 1;               // <= log2(1 + 1/64)
  return m + add;
}

inline int known1(int v) { return std::max(1, v); }

}  // namespace

// lgc of the operands the estimates meet (scalars and constants of the evaluated polynomials,
// the model's constants) is asked for many times per call: the values are kept once computed
int nz_lgc(uint64_t x) {
  static std::mutex mu;
  static std::unordered_map<uint64_t, int> seen;
  std::lock_guard<std::mutex> lock(mu);
  auto it = seen.find(x);
  if (it != seen.end()) return it->second;
  int f, c;
  lg16(x, &f, &c);
  if (seen.size() < (1u << 16)) seen.emplace(x, c);
  return c;
}

int nz_lgf(uint64_t x) {
  int f, c;
  lg16(x, &f, &c);
  return f;
}

void noise_init(bgv_ctx* c) {
  NoiseModel& m = c->nzm;
  const int r = c->prm.r, L = c->prm.L, A = c->alpha, n = c->logN;
  m.fresh = nz_lgc(20 * (uint64_t)c->t_full);
  uint64_t qmin = c->primes[0];
  for (int i = 0; i < L; ++i) qmin = std::min(qmin, c->primes[i]);
  m.q16 = nz_lgf(qmin);
  m.lgp = nz_lgf((uint64_t)c->prm.p);
  m.floor.assign(r + 1, 0);
  m.ks.assign(r + 1, std::vector<int>(L + 1, 0));
  for (int e = 1; e <= r; ++e) {
    const uint64_t t = (uint64_t)c->tpow[e];
    m.floor[e] = nz_lgc(3 * t) - NZ_UNIT + 8 * n;
    for (int lv = 1; lv <= L; ++lv) {
      const int dn = (lv + A - 1) / A;
      m.ks[e][lv] = lsum(nz_lgc(23 * (uint64_t)A * t) + (nz_lgc((uint64_t)dn) + 1) / 2 + 8 * n,
                         nz_lgc(3 * (uint64_t)A * t) + 8 * n);
    }
  }
}

int nz_add(int a, int b) { return a > 0 && b > 0 ? known1(lsum(a, b)) : 0; }

int nz_sum_of(int a, int n) { return a > 0 ? known1(a + nz_lgc((uint64_t)n)) : 0; }

int nz_scalar(int a, int64_t k) { return a > 0 ? known1(a + (k ? nz_lgc((uint64_t)std::llabs(k)) : 0)) : 0; }

int nz_add_const(int a, int64_t k) {
  if (a <= 0) return 0;
  return k ? known1(lsum(a, nz_lgc((uint64_t)std::llabs(k)))) : a;
}

int nz_divide_by_p(const bgv_ctx* c, int a) { return a > 0 ? known1(a - c->nzm.lgp) : 0; }

int nz_switch(const bgv_ctx* c, int a, int t_exp) {
  return a > 0 ? known1(lsum(a - c->nzm.q16, c->nzm.floor[t_exp])) : 0;
}

int nz_tensor(const bgv_ctx* c, int a, int b) { return a > 0 && b > 0 ? a + b + 8 * c->logN + NZ_UNIT : 0; }

int nz_key_switch(const bgv_ctx* c, int a, int t_exp, int level) {
  return a > 0 ? known1(lsum(a, c->nzm.ks[t_exp][level])) : 0;
}

int nz_mul_ms(const bgv_ctx* c, int a, int b, int t_exp, int level) {
  return nz_switch(c, nz_key_switch(c, nz_tensor(c, a, b), t_exp, level), t_exp);
}
