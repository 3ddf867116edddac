// Context creation: prime chain, NTT tables, base-conversion constants, slot
// structure and the coefficient tables of the space-switching polynomials.
#include "ctx.hpp"

#include <cstring>
#include <numeric>

#include "host_nt.hpp"
#include "ops.hpp"

using namespace hnt;

bool hip_ok(bgv_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

// Size classes: 1 MiB, then steps of 1/8 of a power of two (at most 12.5% slack),
// so buffers of neighbouring levels share a class and the cache does not fragment.
static size_t size_class(size_t bytes) {
  const size_t mib = (size_t)1 << 20;
  if (bytes <= mib) return mib;
  size_t p = mib;
  while (p * 2 < bytes) p *= 2;
  const size_t step = p / 8;
  return (bytes + step - 1) / step * step;
}

// A request takes a cached block of its class, else the smallest cached block up to
// twice its class, else a new allocation.  When device memory is short, cached blocks
// are freed largest first only until the allocation fits (every hipFree waits for the
// device, so freeing the whole cache on each miss would serialise the stream).
void* DevPool::get(size_t bytes) {
  bytes = size_class(bytes);
  auto it = free_.lower_bound(bytes);
  if (it != free_.end() && it->first <= 2 * bytes) {
    void* p = it->second;
    free_.erase(it);
    return p;
  }
  void* p = nullptr;
  while (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();  // clear the sticky allocation error
    if (free_.empty() || (pinned && *pinned > 0)) return nullptr;
    auto big = std::prev(free_.end());
    (void)hipFree(big->second);
    auto a = all_.find(big->second);
    if (a != all_.end()) {
      held -= a->second;
      all_.erase(a);
    }
    free_.erase(big);
  }
  all_[p] = bytes;
  held += bytes;
  return p;
}

void DevPool::put(void* p, size_t) {
  if (!p) return;
  auto a = all_.find(p);
  if (a != all_.end()) free_.insert({a->second, p});
}

// Free every cached block that is not in use (after the stream has drained them).
void DevPool::trim() {
  if (pinned && *pinned > 0) return;  // graphs may replay into cached blocks
  for (auto& kv : free_) {
    (void)hipFree(kv.second);
    auto a = all_.find(kv.second);
    if (a != all_.end()) {
      held -= a->second;
      all_.erase(a);
    }
  }
  free_.clear();
}

void DevPool::release() {
  for (auto& a : all_) (void)hipFree(a.first);
  all_.clear();
  free_.clear();
  held = 0;
}

namespace {

// Solve V c = y over Z_m (m a prime power) by Gaussian elimination, pivots units.
bool solve_mod(std::vector<std::vector<int64_t>> A, std::vector<int64_t> y, int64_t m, int64_t p,
               std::vector<int64_t>& out) {
  const int n = (int)y.size();
  for (int col = 0; col < n; ++col) {
    int piv = -1;
    for (int r = col; r < n; ++r)
      if (A[r][col] % p != 0) {
        piv = r;
        break;
      }
    if (piv < 0) return false;
    std::swap(A[piv], A[col]);
    std::swap(y[piv], y[col]);
    const int64_t inv = (int64_t)invmod((uint64_t)((A[col][col] % m + m) % m), (uint64_t)m);
    for (int k = col; k < n; ++k) A[col][k] = (int64_t)((__int128)A[col][k] * inv % m);
    y[col] = (int64_t)((__int128)y[col] * inv % m);
    for (int r = 0; r < n; ++r) {
      if (r == col || A[r][col] == 0) continue;
      const int64_t f = A[r][col];
      for (int k = col; k < n; ++k) A[r][k] = ((A[r][k] - (int64_t)((__int128)f * A[col][k] % m)) % m + m) % m;
      y[r] = ((y[r] - (int64_t)((__int128)f * y[col] % m)) % m + m) % m;
    }
  }
  out = y;
  return true;
}

// unique polynomial of degree < p through (z, f(z)) for every z in Z_p
bool interpolate_fp(int64_t p, const std::vector<int64_t>& zs, const std::vector<int64_t>& vals,
                    std::vector<int64_t>& coeffs) {
  const int n = (int)zs.size();
  std::vector<std::vector<int64_t>> V(n, std::vector<int64_t>(n));
  for (int i = 0; i < n; ++i) {
    int64_t z = ((zs[i] % p) + p) % p, pw = 1;
    for (int k = 0; k < n; ++k) {
      V[i][k] = pw;
      pw = pw * z % p;
    }
  }
  std::vector<int64_t> y(n);
  for (int i = 0; i < n; ++i) y[i] = ((vals[i] % p) + p) % p;
  return solve_mod(V, y, p, p, coeffs);
}

}  // namespace

// Lemma 3 for e >= 3: G_{p,k+1} from G_{p,k}, one digit at a time.  With Q(x) = x^p - x,
// Q(z0 + p y)/p = c(z0) - y (mod p), c(z0) = (z0^p - z0)/p, so Q reaches the digit y.  If
// G_k(z0 + p y) = z0 + p^k E(z0, y) (mod p^(k+1)) -- E of degree <= k in y, found from its
// values at y = 0..k -- then with -E(z0, c - u) = sum_m e_m(z0) u^m and M_m the interpolant
// of e_m over the balanced z0, G_{k+1} = G_k + sum_m p^(k-m) Q^m M_m (mod p^(k+1)).
// Needs k + 1 <= p (distinct sample points) and p^(k+1) < 2^62.
static bool lift_g(int64_t p, int k, const std::vector<int64_t>& G, std::vector<int64_t>& out) {
  if (k + 1 > p) return false;
  int64_t pk = 1;
  for (int i = 0; i < k; ++i) pk *= p;
  const int64_t mod = pk * p;
  if (mod <= 0 || mod > ((int64_t)1 << 62) / p) return false;
  auto mulm = [&](int64_t a, int64_t b) { return (int64_t)((__int128)a * b % mod); };
  auto horner = [&](const std::vector<int64_t>& f, int64_t x) {  // f(x) mod p^(k+1), x in [0, mod)
    int64_t acc = 0;
    for (size_t i = f.size(); i-- > 0;) acc = (mulm(acc, x) + f[i]) % mod;
    return acc;
  };
  auto polymul = [&](const std::vector<int64_t>& a, const std::vector<int64_t>& b) {
    std::vector<int64_t> r(a.size() + b.size() - 1, 0);
    for (size_t i = 0; i < a.size(); ++i)
      if (a[i])
        for (size_t j = 0; j < b.size(); ++j) r[i + j] = (r[i + j] + mulm(a[i], b[j])) % mod;
    return r;
  };
  const int64_t h = (p - 1) / 2;
  std::vector<int64_t> zs, ys;
  for (int64_t z = -h; z <= h; ++z) zs.push_back(z);
  for (int y = 0; y <= k; ++y) ys.push_back(y);
  // binomials mod p (k < p, so they are small)
  std::vector<std::vector<int64_t>> C(k + 1, std::vector<int64_t>(k + 1, 0));
  for (int j = 0; j <= k; ++j) {
    C[j][0] = 1;
    for (int m = 1; m <= j; ++m) C[j][m] = (C[j - 1][m - 1] + (m <= j - 1 ? C[j - 1][m] : 0)) % p;
  }
  std::vector<std::vector<int64_t>> em(k + 1, std::vector<int64_t>(zs.size(), 0));
  for (size_t zi = 0; zi < zs.size(); ++zi) {
    const int64_t z = zs[zi];
    std::vector<int64_t> ev;
    for (int y = 0; y <= k; ++y) {
      const int64_t x = ((z + p * y) % mod + mod) % mod;
      const int64_t v = ((horner(G, x) - z) % mod + mod) % mod;  // divisible by p^k
      if (v % pk != 0) return false;
      ev.push_back(v / pk);
    }
    std::vector<int64_t> E;
    if (!interpolate_fp(p, ys, ev, E)) return false;
    // c(z) = (z^p - z)/p mod p, from z^p mod p^2
    const int64_t t2 = p * p;
    int64_t zz = ((z % t2) + t2) % t2, pw = 1;
    for (int64_t i = 0; i < p; ++i) pw = (int64_t)((__int128)pw * zz % t2);
    const int64_t cz = ((pw - zz) % t2 + t2) % t2 / p;
    // -E(c - u) = sum_m e_m u^m
    for (int j = 0; j <= k; ++j) {
      int64_t cpow = 1;  // c^(j-m), built from m = j downwards
      for (int m = j; m >= 0; --m) {
        int64_t term = E[j] % p * C[j][m] % p * cpow % p;
        if (m & 1) term = (p - term) % p;
        em[m][zi] = ((em[m][zi] - term) % p + p) % p;
        cpow = cpow * cz % p;
      }
    }
  }
  out.assign(G.begin(), G.end());
  for (auto& v : out) v %= mod;
  std::vector<int64_t> Q(p + 1, 0), Qm{1};
  Q[1] = mod - 1;
  Q[p] = 1;
  int64_t pw = pk;  // p^(k-m)
  for (int m = 0; m <= k; ++m) {
    bool any = false;
    for (int64_t v : em[m]) any = any || v != 0;
    if (any) {
      std::vector<int64_t> M;
      if (!interpolate_fp(p, zs, em[m], M)) return false;
      std::vector<int64_t> term = polymul(Qm, M);
      if (out.size() < term.size()) out.resize(term.size(), 0);
      for (size_t i = 0; i < term.size(); ++i) out[i] = (out[i] + mulm(pw, term[i])) % mod;
    }
    Qm = polymul(Qm, Q);
    pw /= p;
  }
  while (out.size() > 1 && out.back() == 0) out.pop_back();
  return true;
}

// F_LT, F_GT: the interpolants over Z_p of [z < 0] and [z > 0] on the balanced representatives.
// G_{p,2} = x^p + p H(x) with H the interpolant of (z - z^p)/p on balanced z:
// then G(z) = z mod p^2 and G'(z) = 0 mod p for every balanced z, so
// G(z0 + p z1) = z0 mod p^2 (Lemma 3 with e = 2, degree p = (e-1)(p-1)+1).
static bool build_poly_tables(bgv_ctx* c) {
  const int64_t p = c->prm.p;
  std::vector<int64_t> zs, lt, gt, phi;
  for (int64_t z = -(p - 1) / 2; z <= (p - 1) / 2; ++z) {
    zs.push_back(z);
    lt.push_back(z < 0 ? 1 : 0);
    gt.push_back(z > 0 ? 1 : 0);
    // (z - z^p)/p mod p computed with exact 128-bit arithmetic on z^p mod p^2
    const int64_t t2 = p * p;
    int64_t zz = ((z % t2) + t2) % t2, pw = 1;
    for (int64_t k = 0; k < p; ++k) pw = (int64_t)((__int128)pw * zz % t2);
    int64_t diff = ((zz - pw) % t2 + t2) % t2;  // divisible by p (Fermat)
    phi.push_back((diff / p) % p);
  }
  if (!interpolate_fp(p, zs, lt, c->flt)) return false;
  if (!interpolate_fp(p, zs, gt, c->fgt)) return false;
  std::vector<int64_t> H;
  if (!interpolate_fp(p, zs, phi, H)) return false;
  const int64_t t2 = p * p;
  c->g2.assign(p + 1, 0);
  for (int64_t k = 0; k < p; ++k) c->g2[k] = (p * H[k]) % t2;
  c->g2[p] = (c->g2[p] + 1) % t2;
  c->gpe.assign(c->prm.r + 1, {});
  if (c->prm.r >= 1) c->gpe[1] = {0, 1};
  if (c->prm.r >= 2) c->gpe[2] = c->g2;
  for (int e = 3; e <= c->prm.r; ++e)
    if (!lift_g(p, e - 1, c->gpe[e - 1], c->gpe[e])) return false;
  return true;
}

static bool build_slots(bgv_ctx* c) {
  const int64_t p = c->prm.p;
  int v = 0;
  for (int64_t x = p - 1; x % 2 == 0; x /= 2) ++v;
  c->ell = 1 << (v - 1);
  if (2 * c->N < (1 << v)) return false;
  c->dslot = c->N / c->ell;
  int64_t zb = 0;
  for (int64_t z = 2; z < p; ++z)
    if ((int64_t)powmod((uint64_t)z, (uint64_t)c->ell, (uint64_t)p) == p - 1) {
      zb = z;
      break;
    }
  if (!zb) return false;
  int64_t e = 1;
  for (int i = 1; i < c->prm.r; ++i) e *= p;
  c->zeta = (int64_t)powmod((uint64_t)zb, (uint64_t)e, (uint64_t)c->t_full);
  const int64_t two_l = 2 * c->ell;
  c->slot_exp.clear();
  for (int rho = 0; rho < 2; ++rho)
    for (int k = 0; k < c->ell / 2; ++k) {
      int64_t ex = (int64_t)powmod(5, (uint64_t)k, (uint64_t)two_l);
      c->slot_exp.push_back(rho == 0 ? ex : (two_l - ex) % two_l);
    }
  return true;
}

template <class T>
static bool upload(bgv_ctx* c, T** dst, const std::vector<T>& v) {
  if (!hip_ok(c, hipMalloc((void**)dst, v.size() * sizeof(T)), "hipMalloc table")) return false;
  return hip_ok(c, hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy table");
}

bgv_status ctx_build(bgv_ctx* c, const bgv_params* prm, hipStream_t stream) {
  c->prm = *prm;
  c->stream = stream;
  c->pool.pinned = &c->graphs_alive;
  if (prm->log_n < 4 || prm->log_n > 16) { c->err = "log_n must be in [4, 16]"; return BGV_E_PARAM; }
  if (prm->p < 5 || prm->p % 4 != 1 || prm->p > 65521) { c->err = "p must be a prime = 1 mod 4 below 2^16"; return BGV_E_PARAM; }
  if (!is_prime((uint64_t)prm->p)) { c->err = "p is not prime"; return BGV_E_PARAM; }
  if (prm->r < 1 || prm->r > 4) { c->err = "r must be in [1, 4]"; return BGV_E_PARAM; }
  if (prm->L < 1 || prm->K < 1 || prm->K > 8 || prm->L + prm->K > 64) { c->err = "need L >= 1, 1 <= K <= 8, L + K <= 64"; return BGV_E_PARAM; }
  c->logN = prm->log_n;
  c->N = 1 << prm->log_n;
  c->alpha = prm->K;
  c->dnum = (prm->L + c->alpha - 1) / c->alpha;
  c->Ltot = prm->L + prm->K;
  c->tpow.assign(prm->r + 1, 1);
  for (int e = 1; e <= prm->r; ++e) c->tpow[e] = c->tpow[e - 1] * prm->p;
  c->t_full = c->tpow[prm->r];
  if (c->t_full >= ((int64_t)1 << 31)) { c->err = "p^r must be below 2^31"; return BGV_E_PARAM; }
  if (!build_slots(c)) { c->err = "ring too small for this p"; return BGV_E_PARAM; }
  const uint64_t M = (uint64_t)(2 * c->N) / gcd((uint64_t)(2 * c->N), (uint64_t)c->t_full) * (uint64_t)c->t_full;
  if (!prime_chain(M, c->Ltot, c->primes)) { c->err = "not enough 50-bit primes = 1 mod lcm(2N, p^r)"; return BGV_E_PARAM; }
  if (!build_poly_tables(c)) { c->err = "polynomial table construction failed"; return BGV_E_PARAM; }

  const int N = c->N, Lt = c->Ltot, L = prm->L, K = prm->K;
  std::vector<PrimeD> pd(Lt);
  std::vector<double> tw((size_t)Lt * N), itw((size_t)Lt * N);
  c->psi.resize(Lt);
  std::vector<uint64_t> pw(N);
  for (int m = 0; m < Lt; ++m) {
    const uint64_t q = c->primes[m];
    const uint64_t psi = min_root_2n(q, (uint64_t)N);
    c->psi[m] = psi;
    pd[m].q = (double)q;
    pd[m].qinv = 1.0 / (double)q;
    pd[m].ninv = (double)invmod((uint64_t)N, q);
    pd[m].pad = 0.0;
    const uint64_t ipsi = invmod(psi, q);
    pw[0] = 1;
    for (int k = 1; k < N; ++k) pw[k] = mulmod(pw[k - 1], psi, q);
    for (int k = 0; k < N; ++k) tw[(size_t)m * N + k] = (double)pw[bitrev((uint32_t)k, c->logN)];
    pw[0] = 1;
    for (int k = 1; k < N; ++k) pw[k] = mulmod(pw[k - 1], ipsi, q);
    for (int k = 0; k < N; ++k) itw[(size_t)m * N + k] = (double)pw[bitrev((uint32_t)k, c->logN)];
  }

  // ModUp tables
  const int A = c->alpha;
  std::vector<double> mu((size_t)(L + 1) * c->dnum * A * (1 + Lt), 0.0);
  for (int lv = 1; lv <= L; ++lv) {
    for (int j = 0; j * A < lv; ++j) {
      const int lo = j * A, hi = std::min(lo + A, lv);
      double* inv = &mu[c->modup_inv_off(lv, j)];
      double* basis = &mu[c->modup_basis_off(lv, j)];
      for (int a = 0; a < hi - lo; ++a) {
        const int i = lo + a;
        const uint64_t qi = c->primes[i];
        uint64_t qh_mod_qi = 1;
        for (int b = lo; b < hi; ++b)
          if (b != i) qh_mod_qi = mulmod(qh_mod_qi, c->primes[b] % qi, qi);
        inv[a] = (double)invmod(qh_mod_qi, qi);
        for (int m = 0; m < Lt; ++m) {
          const uint64_t pm = c->primes[m];
          uint64_t v = 1;
          for (int b = lo; b < hi; ++b)
            if (b != i) v = mulmod(v, c->primes[b] % pm, pm);
          basis[(size_t)a * Lt + m] = (double)v;
        }
      }
    }
  }
  // the fused ModUp's scales: N^-1 Qhat_i^-1 mod q_i (the inverse transform's factor folded in)
  std::vector<double> mus((size_t)(L + 1) * c->dnum * A, 0.0);
  for (int lv = 1; lv <= L; ++lv)
    for (int j = 0; j * A < lv; ++j)
      for (int a = 0; a < std::min(A, lv - j * A); ++a) {
        const uint64_t qi = c->primes[j * A + a];
        const uint64_t inv = (uint64_t)mu[c->modup_inv_off(lv, j) + a];
        mus[((size_t)lv * c->dnum + j) * A + a] = (double)mulmod(inv, invmod((uint64_t)N, qi), qi);
      }
  // ModDown tables: phat_inv [K], phat_mod [K][L], pinv_q [L], pmod_q [L]
  std::vector<double> md((size_t)K + (size_t)K * L + 2 * (size_t)L, 0.0);
  for (int k = 0; k < K; ++k) {
    const uint64_t pk = c->primes[L + k];
    uint64_t v = 1;
    for (int k2 = 0; k2 < K; ++k2)
      if (k2 != k) v = mulmod(v, c->primes[L + k2] % pk, pk);
    md[k] = (double)invmod(v, pk);
    for (int i = 0; i < L; ++i) {
      const uint64_t qi = c->primes[i];
      uint64_t w = 1;
      for (int k2 = 0; k2 < K; ++k2)
        if (k2 != k) w = mulmod(w, c->primes[L + k2] % qi, qi);
      md[K + (size_t)k * L + i] = (double)w;
    }
  }
  for (int i = 0; i < L; ++i) {
    const uint64_t qi = c->primes[i];
    uint64_t P = 1;
    for (int k = 0; k < K; ++k) P = mulmod(P, c->primes[L + k] % qi, qi);
    md[K + (size_t)K * L + i] = (double)invmod(P, qi);
    md[K + (size_t)K * L + L + i] = (double)P;
  }
  // modulus switching: msw[top][i] = q_top^-1 mod q_i
  std::vector<double> msw((size_t)L * L, 0.0);
  for (int top = 0; top < L; ++top)
    for (int i = 0; i < L; ++i)
      if (i != top) msw[(size_t)top * L + i] = (double)invmod(c->primes[top] % c->primes[i], c->primes[i]);
  // repeated switch: mswpi[level][to][i] = prod_{j=to}^{level-1} q_j^-1 mod q_i
  std::vector<double> mswpi((size_t)(L + 1) * (L + 1) * L, 0.0);
  for (int lv = 2; lv <= L; ++lv)
    for (int i = 0; i < lv - 1; ++i) {
      const uint64_t qi = c->primes[i];
      uint64_t v = 1;
      for (int to = lv - 1; to > i; --to) {
        v = mulmod(v, invmod(c->primes[to] % qi, qi), qi);
        mswpi[((size_t)lv * (L + 1) + to) * L + i] = (double)v;
      }
    }
  // t constants [r+1][2][Lt] and the host copy of t^-1
  std::vector<double> tc((size_t)(prm->r + 1) * 2 * Lt);
  c->h_tinv.assign((size_t)(prm->r + 1) * Lt, 0.0);
  c->h_tmod.assign((size_t)(prm->r + 1) * Lt, 0.0);
  for (int e = 0; e <= prm->r; ++e)
    for (int m = 0; m < Lt; ++m) {
      const uint64_t q = c->primes[m];
      const uint64_t tm = (uint64_t)c->tpow[e] % q;
      const double ti = (double)invmod(tm, q);
      tc[((size_t)e * 2 + 0) * Lt + m] = ti;
      tc[((size_t)e * 2 + 1) * Lt + m] = (double)tm;
      c->h_tinv[(size_t)e * Lt + m] = ti;
      c->h_tmod[(size_t)e * Lt + m] = (double)tm;
    }

  // ModDown constants times t P^-1 for the merged switch: mdfold[e][k][i]
  std::vector<double> mdfold((size_t)(prm->r + 1) * K * L, 0.0);
  for (int e = 0; e <= prm->r; ++e)
    for (int k = 0; k < K; ++k)
      for (int i = 0; i < L; ++i) {
        const uint64_t qi = c->primes[i];
        const uint64_t tp = mulmod((uint64_t)c->tpow[e] % qi, (uint64_t)md[K + (size_t)K * L + i], qi);
        mdfold[((size_t)e * K + k) * L + i] = (double)mulmod((uint64_t)md[K + (size_t)k * L + i], tp, qi);
      }
  if (!upload(c, &c->d_prime, pd) || !upload(c, &c->d_tw, tw) || !upload(c, &c->d_itw, itw) ||
      !upload(c, &c->d_modup, mu) || !upload(c, &c->d_moddown, md) || !upload(c, &c->d_msw, msw) ||
      !upload(c, &c->d_mswpi, mswpi) || !upload(c, &c->d_tconst, tc) || !upload(c, &c->d_mdfold, mdfold) ||
      !upload(c, &c->d_modup_scale, mus))
    return BGV_E_DEVICE;
  if (!build_encoder(c)) { c->err = "slot encoder construction failed"; return BGV_E_PARAM; }
  noise_init(c);
  // the allocation-free variant's scratch on this device (looked up once per device)
  c->noalloc_scratch = noalloc_scratch_ptr(&c->device);
  return BGV_OK;
}

void ctx_free(bgv_ctx* c) {
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  c->pool.release();
  for (auto& kv : c->coeff_tabs) (void)hipFree(kv.second);
  c->coeff_tabs.clear();
  void* ptrs[] = {c->d_prime,   c->d_tw,     c->d_itw,    c->d_modup,  c->d_moddown,
                  c->d_msw,     c->d_mswpi,  c->d_tconst, c->d_mdfold, c->d_modup_scale};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
}
