// Operation layer of the library: key switching, modulus switching, encryption,
// decryption, key generation, the Paterson-Stockmeyer evaluator and the
// space-switching composites.  Every device step is a kernel on the context's
// stream; this file only sequences them and manages temporaries.
#include "ops.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "host_nt.hpp"

using hnt::centered;
using hnt::invmod;
using hnt::mulmod;
using hnt::powmod;

Scratch::Scratch(bgv_ctx* cc, size_t words) : c(cc) {
  bytes = words * sizeof(uint64_t);
  d = (uint64_t*)c->pool.get(bytes ? bytes : 8);
  if (!d) throw OpError{BGV_E_OOM};
}

Scratch::~Scratch() {
  if (d) c->pool.put(d, bytes);
}

CipherP new_cipher(bgv_ctx* c, int n, int level, int t_exp) {
  auto p = std::make_shared<Cipher>();
  p->buf = std::make_shared<Scratch>(c, (size_t)n * ct_words(c, level));
  p->v.d = p->buf->d;
  p->v.n = n;
  p->v.level = level;
  p->v.t_exp = t_exp;
  return p;
}

// Algorithmic HBM bytes of the method's steps, in limbs of N words: what a step must read
// and write once (a ciphertext at level l is 2 l limbs), plus the evaluation key of a key
// switch read once per batch call (2 dnum' (l + K) limbs, dnum' = ceil(l / alpha)).  A
// relinearised product reads its two operands and writes its result (6 l; 6 l - 2 when the
// modulus switch after it is merged in), a rotation 4 l, a single modulus switch 4 l - 2.
// Intermediate round trips of an implementation are not counted: this is the floor the
// measured traffic is compared with.
static void algo(bgv_ctx* c, double limbs) { c->stats.algo_bytes += (int64_t)(limbs * c->N * 8.0); }
static double key_limbs(const bgv_ctx* c, int lv) {
  return 2.0 * ((lv + c->alpha - 1) / c->alpha) * (lv + c->prm.K);
}

static void check_hip(bgv_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    throw OpError{BGV_E_DEVICE};
  }
}

void op_copy(bgv_ctx* c, const CtV& in, const CtV& out) {
  if (in.d == out.d) return;
  check_hip(c, hipMemcpyAsync(out.d, in.d, (size_t)in.n * ct_words(c, in.level) * 8, hipMemcpyDeviceToDevice, c->stream),
            "copy");
}

CipherP clone(bgv_ctx* c, const CtV& x) {
  CipherP r = new_cipher(c, x.n, x.level, x.t_exp);
  op_copy(c, x, r->v);
  return r;
}

static LimbMap lm_chain(const bgv_ctx* c, int level) { return LimbMap{level, level, c->prm.L, 0, 1, 0, 0}; }

void op_ntt(bgv_ctx* c, uint64_t* d, int n_polys, int level, bool inverse) {
  lk::ntt(c, d, n_polys * level, lm_chain(c, level), inverse);
}

void op_add_sub(bgv_ctx* c, const CtV& a, const CtV& b, const CtV& out, int op) {
  algo(c, 6.0 * a.level * a.n);
  lk::add_sub(c, a.d, b.d, out.d, a.n, a.level, op, b.n == 1 && a.n > 1, lstride(a), lstride(b));
}

void op_negate(bgv_ctx* c, const CtV& a, const CtV& out) {
  algo(c, 4.0 * a.level * a.n);
  lk::negate(c, a.d, out.d, a.n, a.level);
}

static void scalar_table(const bgv_ctx* c, int64_t k, int level, double* s) {
  for (int i = 0; i < level; ++i) {
    const int64_t q = (int64_t)c->primes[i];
    int64_t v = k % q;
    if (v < 0) v += q;
    s[i] = (double)v;
  }
}

void op_mul_scalar(bgv_ctx* c, const CtV& a, int64_t k, const CtV& out) {
  algo(c, 4.0 * a.level * a.n);
  double s[64];
  scalar_table(c, centered(k, c->tpow[a.t_exp]), a.level, s);
  lk::mul_scalar(c, a.d, out.d, a.n, a.level, s);
}

void op_add_const(bgv_ctx* c, const CtV& a, int64_t k, const CtV& out) {
  algo(c, 4.0 * a.level * a.n);
  double s[64];
  scalar_table(c, centered(k, c->tpow[a.t_exp]), a.level, s);
  lk::add_const(c, a.d, out.d, a.n, a.level, s);
}

void op_divide_by_p(bgv_ctx* c, const CtV& a, const CtV& out) {
  algo(c, 4.0 * a.level * a.n);
  double s[64];
  for (int i = 0; i < a.level; ++i) s[i] = (double)invmod((uint64_t)c->prm.p, c->primes[i]);
  lk::mul_scalar(c, a.d, out.d, a.n, a.level, s);
}

// Hybrid key switching, first half: ModUp of each digit of the polynomial x
// (X = [n][level][N] in evaluation form, left as it is), NTT, and the inner product
// with the key.  Returns u [n][2][level+K][N] in evaluation form.
static std::unique_ptr<Scratch> ks_inner(bgv_ctx* c, const uint64_t* key, const Scratch& X, int n, int level,
                                         const uint64_t* dtop = nullptr, int64_t dtop_ct = 0, int64_t dtop_comp = 0,
                                         double pmod_top = 0.0, int inv_from = -1) {
  const int N = c->N, K = c->prm.K, L = c->prm.L, A = c->alpha;
  const int dn = (level + A - 1) / A, rows = level + K;
  c->stats.key_switches += 1;
  Scratch Y(c, (size_t)n * dn * rows * N);
  Scratch Xc(c, (size_t)n * level * N);
  const bool fused = lk::ntt_fused_inner_ok(c);
  const bool mu_fused = fused && lk::modup_cols_ok(c);
  // a digit's own rows are x as it is: the fused pass reads them from X, the
  // unfused path from a copy in Y
  if (!fused) lk::mod_up_copy_own(c, X.d, (int64_t)level * N, Y.d, n, level);
  if (mu_fused) {
    // x's inverse transform up to its last pass (out of place), then ModUp fused with that
    // last pass and with the first forward pass of every ModUp row
    lk::ntt_inverse_first_pass(c, Xc.d, X.d, n * level, lm_chain(c, level));
    lk::modup_cols(c, Xc.d, Y.d, n, level);
  } else {
    lk::ntt(c, Xc.d, n * level, lm_chain(c, level), true, X.d);  // coefficient form of x, out of place
    lk::mod_up(c, Xc.d, Y.d, n, level);
  }
  std::unique_ptr<Scratch> U(new Scratch(c, (size_t)n * 2 * rows * N));
  if (fused) {
    lk::ntt_pass1_key_inner(c, Y.d, X.d, (int64_t)level * N, key, U->d, n, level, mu_fused, dtop, dtop_ct, dtop_comp,
                            pmod_top, inv_from);
  } else {
    lk::ntt(c, Y.d, n * dn * rows, LimbMap{rows, level, L, A, dn, 0, 0}, false);
    lk::key_inner(c, Y.d, key, U->d, n, level);
  }
  return U;
}

// The special rows of u [n][2][level+K][N] to coefficient form, in place.
static void special_rows_coeff(bgv_ctx* c, Scratch& U, int n, int level) {
  const int K = c->prm.K, rows = level + K;
  LimbMap lm{K, 0, c->prm.L, 0, 1, 0, 0};
  lm.grp = K;
  lm.grp_stride = rows;
  lm.grp_first = level;
  lk::ntt(c, U.d, n * 2 * K, lm, true);
}

// Hybrid key switching of X under `key`; out[b][comp] = add[b][comp] (comp < add_comps) + switched[comp].
static void key_switch(bgv_ctx* c, const uint64_t* key, Scratch& X, int n, int level, int t_exp, const uint64_t* add,
                       int64_t add_stride, int add_comps, uint64_t* out) {
  const int N = c->N, rows = level + c->prm.K;
  auto U = ks_inner(c, key, X, n, level);
  special_rows_coeff(c, *U, n, level);
  Scratch DL(c, (size_t)n * 2 * level * N);
  lk::mod_down_delta(c, U->d + (size_t)level * N, (int64_t)rows * N, DL.d, n, level, t_exp);
  op_ntt(c, DL.d, n * 2, level, false);
  lk::mod_down_final(c, U->d, DL.d, add, add_comps == 2 ? add_stride : -add_stride, out, n, level, t_exp);
}

// Relinearisation of a tensor triple followed by one modulus switch, with the switch
// merged into ModDown: both corrections are formed in coefficient form and go through one
// NTT (the transform is linear over every Z_q_i, so the words equal those of the
// relinearised triple followed by the separate switch).  D [n][2][lv][N] holds d0, d1 and
// X [n][lv][N] holds d2; the top rows of u and d are dropped by the switch, so they are
// brought to coefficient form in place.
static void relin_ms(bgv_ctx* c, const bgv_keys* keys, Scratch& D, Scratch& X, int n, int lv, int t_exp,
                     const CtV& out) {
  const int N = c->N, K = c->prm.K;
  const int rows = lv + K;
  // With the fused inner product, d's top row joins u's as u_top + P d_top (P mod the top
  // prime), so it needs no inverse transform of its own; otherwise it is transformed apart.
  const bool fold_top = lk::ntt_fused_inner_ok(c);
  const uint64_t* dtop = D.d + (size_t)(lv - 1) * N;
  double pmod_top = 0.0;
  if (fold_top) {
    const uint64_t qt = c->primes[lv - 1];
    uint64_t pm = 1;
    for (int k = 0; k < K; ++k) pm = mulmod(pm, c->primes[c->prm.L + k] % qt, qt);
    pmod_top = (double)pm;
  }
  // With the fused inner product, that pass also runs the first pass of the inverse transform
  // of u's top and special rows before storing them.
  auto U = fold_top ? ks_inner(c, keys->relin, X, n, lv, dtop, (int64_t)2 * lv * N, (int64_t)lv * N, pmod_top, lv - 1)
                    : ks_inner(c, keys->relin, X, n, lv);
  // u's top row and its special rows are the K + 1 consecutive rows lv-1 .. lv+K-1
  // of every polynomial: one inverse transform brings them all to coefficient form
  LimbMap ut{K + 1, 1, c->prm.L, 0, 1, lv - 1, 0};
  ut.grp = K + 1;
  ut.grp_stride = rows;
  ut.grp_first = lv - 1;
  // with the fused ModDown, the last inverse pass of those rows, the correction and its first
  // forward pass are one kernel
  const bool md_fused = fold_top && lk::moddown_cols_ok(c, n);
  if (!md_fused) {
    if (fold_top)
      lk::ntt_inverse_last_pass(c, U->d, 2 * n * (K + 1), ut);
    else
      lk::ntt(c, U->d, 2 * n * (K + 1), ut, true);
  }
  if (!fold_top) {
    LimbMap top{1, 1, c->prm.L, 0, 1, lv - 1, 0};
    top.grp = 1;
    top.grp_stride = lv;
    top.grp_first = lv - 1;
    lk::ntt(c, D.d, 2 * n, top, true);  // d tops
  }
  Scratch E(c, (size_t)n * 2 * (lv - 1) * N);
  if (md_fused)
    lk::moddown_cols(c, U->d, E.d, n, lv, t_exp);
  else
    lk::ms_corr(c, U->d + (size_t)lv * N, (int64_t)rows * N, U->d + (size_t)(lv - 1) * N, (int64_t)rows * N,
                fold_top ? nullptr : dtop, (int64_t)lv * N, E.d, n, lv, t_exp);
  // forward NTT of e with the final step in its last pass:
  // out_i = (d_i - e_i + u_i P^-1) q_top^-1 for i < level-1
  lk::NttEpi ep{};
  ep.a = D.d;
  ep.a_cc = (int64_t)lv * N;
  ep.b = U->d;
  ep.b_cc = (int64_t)rows * N;
  ep.sb = c->d_moddown + K + (size_t)K * c->prm.L;  // P^-1 mod q_i
  ep.qt = c->d_msw + (size_t)(lv - 1) * c->prm.L;   // q_top^-1 mod q_i
  ep.out = out.d;
  ep.rows = lv - 1;
  if (md_fused)
    lk::ntt_forward_last_pass(c, E.d, n * 2 * (lv - 1), lm_chain(c, lv - 1), &ep);
  else
    lk::ntt(c, E.d, n * 2 * (lv - 1), lm_chain(c, lv - 1), false, nullptr, &ep);
}

// Relinearised product followed by one modulus switch.
void op_mul_ms(bgv_ctx* c, const bgv_keys* keys, const CtV& a, const CtV& b, const CtV& out) {
  const int n = a.n, lv = a.level, N = c->N;
  if (lv < 2) throw OpError{BGV_E_LEVEL};
  algo(c, (6.0 * lv - 2.0) * n + key_limbs(c, lv));
  Scratch D(c, (size_t)n * 2 * lv * N), X(c, (size_t)n * lv * N);
  lk::tensor(c, a.d, b.d, D.d, X.d, n, lv, b.n == 1 && n > 1, lstride(a), lstride(b));
  relin_ms(c, keys, D, X, n, lv, a.t_exp, out);
}

static CipherP ev_lower(bgv_ctx* c, const CipherP& x, int level);
static CipherP ev_drop(bgv_ctx* c, const CipherP& x, int level);
static CipherP ev_scalar(bgv_ctx* c, const CipherP& x0, int64_t k);

static int lazy_level(const std::vector<std::pair<CipherP, CipherP>>& pairs) {
  int lv = 1 << 30;
  for (const auto& pr : pairs) lv = std::min(lv, std::min(pr.first->v.level, pr.second->v.level));
  return lv;
}

// sum_j a_j b_j relinearised once: every operand brought to the lowest level among the
// pairs, the tensor products accumulated, one key switch and one modulus switch.  Addends
// (k, x): k x for each, in their order, x at that level or above and brought down by dropping
// limbs, join (d0, d1) before the key switch, so the one modulus switch also divides their noise.
static CipherP ev_lazy_products(bgv_ctx* c, const bgv_keys* k, const std::vector<std::pair<CipherP, CipherP>>& pairs,
                                const std::vector<std::pair<int64_t, CipherP>>& addends = {}) {
  int lv = 1 << 30, n = 1;
  for (const auto& pr : pairs) {
    lv = std::min(lv, std::min(pr.first->v.level, pr.second->v.level));
    n = std::max(n, std::max(pr.first->v.n, pr.second->v.n));
    if (pr.first->v.t_exp != pairs[0].first->v.t_exp || pr.second->v.t_exp != pairs[0].first->v.t_exp)
      throw OpError{BGV_E_PTXT_MOD};
  }
  if (lv < 2) throw OpError{BGV_E_LEVEL};
  const int t_exp = pairs[0].first->v.t_exp, N = c->N;
  algo(c, (4.0 * lv * pairs.size() + 2.0 * (lv - 1)) * n + key_limbs(c, lv));
  Scratch D(c, (size_t)n * 2 * lv * N), X(c, (size_t)n * lv * N);
  int nz = 0;  // the tensor estimates accumulated in the pairs' order
  // the pairs' tensor products summed in passes of at most TS_MAX pairs (each operand read once)
  for (size_t s0 = 0; s0 < pairs.size(); s0 += lk::TS_MAX) {
    const int np = (int)std::min<size_t>(lk::TS_MAX, pairs.size() - s0);
    std::vector<CipherP> keep;
    lk::TensorPairs tp{};
    for (int t = 0; t < np; ++t) {
      CipherP a = ev_lower(c, pairs[s0 + t].first, lv);
      CipherP b = ev_lower(c, pairs[s0 + t].second, lv);
      const int tz = nz_tensor(c, a->v.nz, b->v.nz);
      nz = s0 + t == 0 ? tz : nz_add(nz, tz);
      if (a->v.n == 1 && n > 1) std::swap(a, b);
      tp.a[t] = a->v.d;
      tp.b[t] = b->v.d;
      tp.sa[t] = lstride(a->v);
      tp.sb[t] = lstride(b->v);
      tp.bb[t] = b->v.n == 1 && n > 1;
      keep.push_back(a);
      keep.push_back(b);
    }
    c->stats.max_tensor_pairs = std::max(c->stats.max_tensor_pairs, np);
    lk::tensor_sum(c, tp, np, D.d, X.d, n, lv, s0 > 0);
  }
  for (const auto& ad : addends) {
    if (ad.second->v.level < lv || ad.second->v.t_exp != t_exp || (ad.second->v.n != n && ad.second->v.n != 1))
      throw OpError{BGV_E_ARG};
    const CipherP xd = ev_drop(c, ad.second, lv);
    const CipherP term = ad.first == 1 ? xd : ev_scalar(c, xd, ad.first);
    CtV dv;
    dv.d = D.d;
    dv.n = n;
    dv.level = lv;
    dv.t_exp = t_exp;
    op_add_sub(c, dv, term->v, dv, 0);  // (d0, d1) += term, a single ciphertext broadcast
    nz = nz_add(nz, term->v.nz);
  }
  CipherP r = new_cipher(c, n, lv - 1, t_exp);
  relin_ms(c, k, D, X, n, lv, t_exp, r->v);
  r->v.nz = nz_switch(c, nz_key_switch(c, nz, t_exp, lv), t_exp);
  return r;
}

void op_mul_relin(bgv_ctx* c, const bgv_keys* keys, const CtV& a, const CtV& b, const CtV& out) {
  const int n = a.n, lv = a.level, N = c->N;
  algo(c, 6.0 * lv * n + key_limbs(c, lv));
  Scratch D(c, (size_t)n * 2 * lv * N), X(c, (size_t)n * lv * N);
  lk::tensor(c, a.d, b.d, D.d, X.d, n, lv, b.n == 1 && n > 1);
  key_switch(c, keys->relin, X, n, lv, a.t_exp, D.d, (int64_t)2 * lv * N, 2, out.d);
}

int galois_elt(const bgv_ctx* c, int step) {
  const uint64_t two_n = 2 * (uint64_t)c->N;
  if (step == BGV_ROW_SWAP) return (int)(two_n - 1);
  const int half = c->ell / 2;
  int s = ((step % half) + half) % half;
  return (int)powmod(5, (uint64_t)s, two_n);
}

void op_rotate(bgv_ctx* c, const bgv_keys* keys, const CtV& in, int g, const CtV& out) {
  const int n = in.n, lv = in.level, N = c->N;
  auto it = keys->galois.find(g);
  if (it == keys->galois.end()) throw OpError{BGV_E_NOKEY};
  algo(c, 4.0 * lv * n + key_limbs(c, lv));
  Scratch R(c, (size_t)n * lv * N), X(c, (size_t)n * lv * N);
  const int64_t st = (int64_t)2 * lv * N;
  lk::automorph(c, in.d, st, R.d, (int64_t)lv * N, n, lv, g);              // X -> X^g on c0
  lk::automorph(c, in.d + (size_t)lv * N, st, X.d, (int64_t)lv * N, n, lv, g);  // and on c1
  key_switch(c, it->second, X, n, lv, in.t_exp, R.d, (int64_t)lv * N, 1, out.d);
}

// Single modulus switch with caller-provided scratch: T [n][2][N] receives the top limbs
// (coefficient form), W [n][2][level-1][N] the correction w and, for an in-place call, the
// result before it is copied back.  Every word of T and W is written before it is read.
void op_mod_switch_with(bgv_ctx* c, const CtV& in, const CtV& out, uint64_t* T, uint64_t* W) {
  const int n = in.n, lv = in.level, N = c->N;
  if (lv < 2) throw OpError{BGV_E_LEVEL};
  c->stats.rescale_drops += 1;
  algo(c, (4.0 * lv - 2.0) * n);
  check_hip(c,
            hipMemcpy2DAsync(T, (size_t)N * 8, in.d + (size_t)(lv - 1) * N, (size_t)lv * N * 8, (size_t)N * 8,
                             (size_t)n * 2, hipMemcpyDeviceToDevice, c->stream),
            "gather top");
  lk::ntt(c, T, n * 2, LimbMap{1, 1, c->prm.L, 0, 1, lv - 1, 0}, true);
  lk::msw_w(c, T, W, n, lv, in.t_exp);
  // forward NTT of w with the final step in its last pass:
  // out_i = (x_i - t w_i) q_top^-1 for i < level-1
  lk::NttEpi ep{};
  ep.a = in.d;
  ep.a_cc = (int64_t)lv * N;
  ep.sv = c->d_tconst + ((size_t)2 * in.t_exp + 1) * c->Ltot;  // t mod q_i
  ep.qt = c->d_msw + (size_t)(lv - 1) * c->prm.L;              // q_top^-1 mod q_i
  ep.out = out.d == in.d ? W : out.d;  // in place: the result goes through w
  ep.rows = lv - 1;
  lk::ntt(c, W, n * 2 * (lv - 1), lm_chain(c, lv - 1), false, nullptr, &ep);
  if (out.d == in.d)
    check_hip(c, hipMemcpyAsync(out.d, W, (size_t)n * 2 * (lv - 1) * N * 8, hipMemcpyDeviceToDevice, c->stream),
              "copy");
}

void op_mod_switch(bgv_ctx* c, const CtV& in, const CtV& out) {
  const int n = in.n, lv = in.level, N = c->N;
  if (lv < 2) throw OpError{BGV_E_LEVEL};
  Scratch T(c, (size_t)n * 2 * N);
  Scratch W(c, (size_t)n * 2 * (lv - 1) * N);
  op_mod_switch_with(c, in, out, T.d, W.d);
}

void op_mod_switch_to(bgv_ctx* c, const CtV& in, int to, const CtV& out) {
  const int n = in.n, lv = in.level, N = c->N;
  if (to > lv || to < 1) throw OpError{BGV_E_LEVEL};
  if (to == lv) {
    op_copy(c, in, out);
    return;
  }
  if (to == lv - 1) {
    op_mod_switch(c, in, out);
    return;
  }
  c->stats.rescale_drops += lv - to;
  algo(c, (2.0 * lv + 2.0 * to) * n);
  // At most 16 drops per step.  A step brings only the dropped limbs to coefficient
  // form, forms the combined correction e for the kept ones, and finishes in the epilogue
  // of e's forward NTT: out_i = (c_i - e_i) prod q_dropped^-1 with c in evaluation form.
  // Chained steps are the same sequence of single-prime drops.
  const int L = c->prm.L;
  const uint64_t* src = in.d;
  std::unique_ptr<Scratch> cur_buf;
  int cur = lv;
  while (cur > to) {
    const int nxt = std::max(to, cur - 16);
    const int nd = cur - nxt;
    Scratch T(c, (size_t)n * 2 * nd * N);
    LimbMap tm{nd, nd, L, 0, 1, nxt, 0};
    tm.sgrp = nd;
    tm.sgrp_stride = cur;
    tm.sgrp_first = nxt;
    lk::ntt(c, T.d, n * 2 * nd, tm, true, src);  // the dropped rows of src, out of place
    std::unique_ptr<Scratch> E(new Scratch(c, (size_t)n * 2 * nxt * N));
    lk::msw_corr(c, T.d, E->d, n, cur, nxt, in.t_exp);
    lk::NttEpi ep{};
    ep.a = src;
    ep.a_cc = (int64_t)cur * N;
    ep.qt = c->d_mswpi + ((size_t)cur * (L + 1) + nxt) * L;
    ep.rows = nxt;
    // the result goes to out unless it is the input's own buffer (rows at another
    // stride) or an intermediate step; then it stays in e, transformed in place
    const bool direct = nxt == to && out.d != in.d;
    ep.out = direct ? out.d : E->d;
    lk::ntt(c, E->d, n * 2 * nxt, lm_chain(c, nxt), false, nullptr, &ep);
    cur_buf = std::move(E);  // the previous step's buffer goes back to the pool: its readers are enqueued
    src = cur_buf->d;
    cur = nxt;
    if (direct) return;
  }
  check_hip(c, hipMemcpyAsync(out.d, src, (size_t)n * 2 * to * N * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
}

// ------------------------------------------------------------------ encoding

// Slot encoder: the inverse of the Vandermonde matrix V[j][k] = zeta_j^k over
// Z_{p^r}, found by Gauss-Jordan elimination (the slot roots are distinct mod p,
// so every pivot is a unit).  encode(v) = Vinv v gives the coefficients of M(Y).
bool build_encoder(bgv_ctx* c) {
  const int l = c->ell;
  const int64_t t = c->t_full, p = c->prm.p;
  std::vector<std::vector<int64_t>> A(l, std::vector<int64_t>(2 * l, 0));
  for (int j = 0; j < l; ++j) {
    const int64_t z = (int64_t)powmod((uint64_t)c->zeta, (uint64_t)c->slot_exp[j], (uint64_t)t);
    int64_t pw = 1;
    for (int k = 0; k < l; ++k) {
      A[j][k] = pw;
      pw = (int64_t)((__int128)pw * z % t);
    }
    A[j][l + j] = 1;
  }
  for (int col = 0; col < l; ++col) {
    int piv = -1;
    for (int r = col; r < l; ++r)
      if (A[r][col] % p) {
        piv = r;
        break;
      }
    if (piv < 0) return false;
    std::swap(A[piv], A[col]);
    const int64_t inv = (int64_t)invmod((uint64_t)A[col][col], (uint64_t)t);
    for (int k = 0; k < 2 * l; ++k) A[col][k] = (int64_t)((__int128)A[col][k] * inv % t);
    for (int r = 0; r < l; ++r) {
      if (r == col || A[r][col] == 0) continue;
      const int64_t f = A[r][col];
      for (int k = 0; k < 2 * l; ++k) A[r][k] = ((A[r][k] - (int64_t)((__int128)f * A[col][k] % t)) % t + t) % t;
    }
  }
  // the inverse sits in the right half: row k of Vinv maps slot values to coefficient k
  std::vector<int64_t>& Vinv = c->encoder;
  Vinv.assign((size_t)l * l, 0);
  for (int k = 0; k < l; ++k)
    for (int j = 0; j < l; ++j) Vinv[(size_t)k * l + j] = A[k][l + j];
  return true;
}

static void encode_slots(const bgv_ctx* c, const uint64_t* v, int64_t* m) {
  const int l = c->ell;
  const int64_t t = c->t_full;
  std::memset(m, 0, sizeof(int64_t) * c->N);
  for (int k = 0; k < l; ++k) {
    __int128 acc = 0;
    for (int j = 0; j < l; ++j) acc += (__int128)c->encoder[(size_t)k * l + j] * (int64_t)(v[j] % (uint64_t)t);
    m[(size_t)k * c->dslot] = centered((int64_t)(acc % t), t);
  }
}

bgv_status op_encrypt(bgv_ctx* c, const int8_t* s, const uint64_t* slots, const uint64_t* c1, const int32_t* e,
                      const CtV& out) {
  const int n = out.n, L = c->prm.L, N = c->N;
  std::vector<int64_t> me((size_t)n * N), s64(N);
  for (int b = 0; b < n; ++b) {
    encode_slots(c, slots + (size_t)b * c->ell, &me[(size_t)b * N]);
    for (int k = 0; k < N; ++k) me[(size_t)b * N + k] += c->t_full * (int64_t)e[(size_t)b * N + k];
  }
  for (int k = 0; k < N; ++k) s64[k] = s[k];
  Scratch dme(c, (size_t)n * N), ds(c, (size_t)N), M(c, (size_t)n * L * N), S(c, (size_t)L * N),
      C1(c, (size_t)n * L * N);
  check_hip(c, hipMemcpyAsync(dme.d, me.data(), me.size() * 8, hipMemcpyHostToDevice, c->stream), "upload");
  check_hip(c, hipMemcpyAsync(ds.d, s64.data(), s64.size() * 8, hipMemcpyHostToDevice, c->stream), "upload");
  check_hip(c, hipMemcpyAsync(C1.d, c1, (size_t)n * L * N * 8, hipMemcpyHostToDevice, c->stream), "upload");
  lk::from_signed(c, (const int64_t*)dme.d, M.d, n, L, lm_chain(c, L));
  op_ntt(c, M.d, n, L, false);
  lk::from_signed(c, (const int64_t*)ds.d, S.d, 1, L, lm_chain(c, L));
  op_ntt(c, S.d, 1, L, false);
  op_ntt(c, C1.d, n, L, false);
  lk::enc_combine(c, M.d, C1.d, S.d, out.d, n);
  check_hip(c, hipStreamSynchronize(c->stream), "sync");
  return BGV_OK;
}

bgv_status op_decrypt(bgv_ctx* c, const int8_t* s, const CtV& in, uint64_t* slots, uint8_t* nonconst) {
  const int n = in.n, lv = in.level, N = c->N;
  std::vector<int64_t> s64(N);
  for (int k = 0; k < N; ++k) s64[k] = s[k];
  Scratch ds(c, (size_t)N), S(c, (size_t)lv * N), V(c, (size_t)n * lv * N);
  check_hip(c, hipMemcpyAsync(ds.d, s64.data(), s64.size() * 8, hipMemcpyHostToDevice, c->stream), "upload");
  lk::from_signed(c, (const int64_t*)ds.d, S.d, 1, lv, lm_chain(c, lv));
  op_ntt(c, S.d, 1, lv, false);
  lk::phase(c, in.d, S.d, V.d, n, lv);
  op_ntt(c, V.d, n, lv, true);
  std::vector<uint64_t> hv((size_t)n * lv * N);
  check_hip(c, hipMemcpyAsync(hv.data(), V.d, hv.size() * 8, hipMemcpyDeviceToHost, c->stream), "download");
  check_hip(c, hipStreamSynchronize(c->stream), "sync");

  // CRT to the centered integer mod Q_lv, reduced mod t: with y_i = [v_i Qhat_i^-1]_{q_i},
  // V = sum y_i Qhat_i - k Q where k = round(sum y_i / q_i) (V is tiny against Q).
  const int64_t t = c->tpow[in.t_exp];
  std::vector<uint64_t> qhinv(lv);
  std::vector<int64_t> qh_t(lv);
  int64_t Q_t = 1;
  for (int i = 0; i < lv; ++i) {
    const uint64_t qi = c->primes[i];
    uint64_t qh = 1;
    int64_t qht = 1;
    for (int j = 0; j < lv; ++j)
      if (j != i) {
        qh = mulmod(qh, c->primes[j] % qi, qi);
        qht = (int64_t)((__int128)qht * (int64_t)(c->primes[j] % (uint64_t)t) % t);
      }
    qhinv[i] = invmod(qh, qi);
    qh_t[i] = qht;
    Q_t = (int64_t)((__int128)Q_t * (int64_t)(qi % (uint64_t)t) % t);
  }
  std::vector<int64_t> m(N);
  const int l = c->ell, d = c->dslot;
  for (int b = 0; b < n; ++b) {
    for (int k = 0; k < N; ++k) {
      long double frac = 0.0L;
      __int128 acc = 0;
      for (int i = 0; i < lv; ++i) {
        const uint64_t qi = c->primes[i];
        const uint64_t y = mulmod(hv[((size_t)b * lv + i) * N + k], qhinv[i], qi);
        frac += (long double)y / (long double)qi;
        acc += (__int128)(int64_t)(y % (uint64_t)t) * qh_t[i];
      }
      const int64_t kk = (int64_t)llroundl(frac);
      __int128 val = (acc - (__int128)(kk % t) * Q_t) % t;
      if (val < 0) val += t;
      m[k] = (int64_t)val;
    }
    // slot j = m(X) mod (X^d - zeta_j): fold with powers of zeta_j
    for (int j = 0; j < l; ++j) {
      const int64_t z = (int64_t)powmod((uint64_t)(c->zeta % t), (uint64_t)c->slot_exp[j], (uint64_t)t);
      bool nc = false;
      int64_t val0 = 0;
      for (int bb = 0; bb < d; ++bb) {
        __int128 acc = 0;
        int64_t zp = 1;
        for (int a = 0; a < l; ++a) {
          acc += (__int128)m[(size_t)a * d + bb] * zp;
          zp = (int64_t)((__int128)zp * z % t);
        }
        const int64_t r = (int64_t)(acc % t);
        if (bb == 0) val0 = r;
        else if (r != 0) nc = true;
        if (!nonconst && bb == 0) break;
      }
      slots[(size_t)b * l + j] = (uint64_t)val0;
      if (nonconst) nonconst[(size_t)b * l + j] = nc ? 1 : 0;
    }
  }
  return BGV_OK;
}

bgv_status op_keygen(bgv_ctx* c, const int8_t* s, const uint64_t* a, const int32_t* e, const std::vector<int>& gal,
                     bgv_keys* keys) {
  const int N = c->N, Lt = c->Ltot, dn = c->dnum;
  std::vector<int64_t> s64(N);
  for (int k = 0; k < N; ++k) s64[k] = s[k];
  Scratch ds(c, (size_t)N), S(c, (size_t)Lt * N), Sp(c, (size_t)Lt * N), A(c, (size_t)dn * Lt * N),
      E(c, (size_t)dn * Lt * N), de(c, (size_t)dn * N);
  check_hip(c, hipMemcpyAsync(ds.d, s64.data(), s64.size() * 8, hipMemcpyHostToDevice, c->stream), "upload");
  lk::from_signed(c, (const int64_t*)ds.d, S.d, 1, Lt, lm_chain(c, Lt));
  op_ntt(c, S.d, 1, Lt, false);
  const size_t key_words = (size_t)dn * 2 * Lt * N;
  std::vector<int64_t> e64((size_t)dn * N);
  const int n_keys = 1 + (int)gal.size();
  for (int kidx = 0; kidx < n_keys; ++kidx) {
    if (kidx == 0) {
      lk::mul_pointwise(c, S.d, S.d, Sp.d, Lt, lm_chain(c, Lt), 0);
    } else {
      lk::automorph(c, S.d, 0, Sp.d, 0, 1, Lt, gal[kidx - 1]);
    }
    check_hip(c, hipMemcpyAsync(A.d, a + (size_t)kidx * dn * Lt * N, (size_t)dn * Lt * N * 8, hipMemcpyHostToDevice,
                                c->stream),
              "upload");
    op_ntt(c, A.d, dn, Lt, false);
    for (size_t i = 0; i < e64.size(); ++i) e64[i] = e[(size_t)kidx * dn * N + i];
    check_hip(c, hipMemcpyAsync(de.d, e64.data(), e64.size() * 8, hipMemcpyHostToDevice, c->stream), "upload");
    lk::from_signed(c, (const int64_t*)de.d, E.d, dn, Lt, lm_chain(c, Lt));
    op_ntt(c, E.d, dn, Lt, false);
    uint64_t* kd = nullptr;
    check_hip(c, hipMalloc((void**)&kd, key_words * 8), "key alloc");
    lk::key_combine(c, A.d, S.d, E.d, Sp.d, kd, dn);
    keys->bytes += (int64_t)key_words * 8;
    if (kidx == 0) keys->relin = kd;
    else keys->galois[gal[kidx - 1]] = kd;
    check_hip(c, hipStreamSynchronize(c->stream), "sync");  // host staging buffers are reused
  }
  return BGV_OK;
}

// ------------------------------------------------------------------ evaluator


// x brought to `level` by single-prime rescaling switches
CipherP ev_align(bgv_ctx* c, const CipherP& x, int level) {
  if (x->v.level == level) return x;
  if (level > x->v.level || level < 1) throw OpError{BGV_E_LEVEL};
  const CipherP src = ev_materialize(c, x);  // the switch reads whole polynomials
  CipherP r = new_cipher(c, x->v.n, level, x->v.t_exp);
  op_mod_switch_to(c, src->v, level, r->v);
  int nz = x->v.nz;
  for (int l = x->v.level; l > level; --l) nz = nz_switch(c, nz, x->v.t_exp);
  r->v.nz = nz;
  return r;
}

static CipherP with_t(const CipherP& x, int t_exp) {
  auto r = std::make_shared<Cipher>();
  r->buf = x->buf;
  r->v = x->v;
  r->v.t_exp = t_exp;
  return r;
}

// The ciphertext reduced modulo its first `level` primes: the top limbs are dropped
// without rescaling (the decryption relation holds modulo every divisor of the
// modulus, and the primes are 1 mod t, so the message is unchanged).  The noise
// keeps its size.  The result is a view of x's lower limbs (no copy, polynomial stride
// x's); the tensor kernels, the inner sums and additions read views, and
// ev_materialize copies one for the other operations.
static CipherP ev_drop(bgv_ctx* c, const CipherP& x, int level) {
  if (x->v.level == level) return x;
  if (level > x->v.level || level < 1) throw OpError{BGV_E_LEVEL};
  c->stats.limb_drops += 1;
  auto r = std::make_shared<Cipher>();
  r->buf = x->buf;
  r->v = x->v;
  r->v.level = level;
  r->v.stride = lstride(x->v);
  return r;
}

CipherP ev_materialize(bgv_ctx* c, const CipherP& x) {
  if (lstride(x->v) == x->v.level) return x;
  CipherP r = new_cipher(c, x->v.n, x->v.level, x->v.t_exp);
  r->v.nz = x->v.nz;
  const size_t N = c->N;
  check_hip(c,
            hipMemcpy2DAsync(r->v.d, (size_t)x->v.level * N * 8, x->v.d, (size_t)lstride(x->v) * N * 8,
                             (size_t)x->v.level * N * 8, (size_t)x->v.n * 2, hipMemcpyDeviceToDevice, c->stream),
            "copy the kept limbs");
  return r;
}

// x brought to `level`.  In the basic schedule, or without a noise estimate, by
// single-prime rescaling switches.  In the fast schedule by the estimate: while it is more
// than NZ_SLACK above the floor a switch leaves, one switch of the top prime; the limbs
// left above `level` are dropped without rescaling (their noise is then within NZ_SLACK
// of what further switches would leave).
static int lower_switches(const bgv_ctx* c, const CipherP& x, int level) {
  const int te = x->v.t_exp, limit = c->nzm.floor[te] + NZ_SLACK;
  int m = 0;
  for (int e = x->v.nz; m < x->v.level - level && e > limit; ++m) e = nz_switch(c, e, te);
  return m;
}

static CipherP ev_lower(bgv_ctx* c, const CipherP& x, int level) {
  if (x->v.level == level) return x;
  if (level > x->v.level || level < 1) throw OpError{BGV_E_LEVEL};
  if (c->schedule == BGV_SCHED_BASIC || x->v.nz <= 0) return ev_align(c, x, level);
  const int m = lower_switches(c, x, level);
  const CipherP y = m ? ev_align(c, x, x->v.level - m) : x;
  return ev_drop(c, y, level);
}

// ev_lower for an operand lowered to several levels: its switched form (the switches depend
// only on its estimate and level) is formed once and kept in `done`
typedef std::map<std::pair<const Cipher*, int>, CipherP> SwitchedForms;
static CipherP ev_lower_shared(bgv_ctx* c, const CipherP& x, int level, SwitchedForms& done) {
  if (x->v.level == level || c->schedule == BGV_SCHED_BASIC || x->v.nz <= 0) return ev_lower(c, x, level);
  if (level > x->v.level || level < 1) throw OpError{BGV_E_LEVEL};
  const int m = lower_switches(c, x, level);
  if (m == 0) return ev_drop(c, x, level);
  const auto key = std::make_pair(x.get(), m);
  auto it = done.find(key);
  if (it == done.end()) it = done.emplace(key, ev_align(c, x, x->v.level - m)).first;
  return ev_drop(c, it->second, level);
}

// a * b relinearised and switched down one prime, each operand first brought to the lower level
CipherP ev_mul(bgv_ctx* c, const bgv_keys* k, const CipherP& a, const CipherP& b) {
  const int lv = std::min(a->v.level, b->v.level);
  if (lv < 2) throw OpError{BGV_E_LEVEL};
  if (a->v.t_exp != b->v.t_exp) throw OpError{BGV_E_PTXT_MOD};
  CipherP a2 = ev_lower(c, a, lv), b2 = ev_lower(c, b, lv);
  const int n = std::max(a->v.n, b->v.n);
  CipherP r = new_cipher(c, n, lv - 1, a->v.t_exp);
  if (a2->v.n == 1 && n > 1) op_mul_ms(c, k, b2->v, a2->v, r->v);
  else op_mul_ms(c, k, a2->v, b2->v, r->v);
  r->v.nz = nz_mul_ms(c, a2->v.nz, b2->v.nz, a->v.t_exp, lv);
  return r;
}

CipherP ev_add(bgv_ctx* c, const CipherP& a, const CipherP& b) {
  const int lv = std::min(a->v.level, b->v.level);
  if (a->v.t_exp != b->v.t_exp) throw OpError{BGV_E_PTXT_MOD};
  CipherP a2 = ev_lower(c, a, lv), b2 = ev_lower(c, b, lv);
  const int n = std::max(a->v.n, b->v.n);
  CipherP r = new_cipher(c, n, lv, a->v.t_exp);
  if (a2->v.n == 1 && n > 1) op_add_sub(c, b2->v, a2->v, r->v, 0);
  else op_add_sub(c, a2->v, b2->v, r->v, 0);
  r->v.nz = nz_add(a2->v.nz, b2->v.nz);
  return r;
}

static CipherP ev_scalar(bgv_ctx* c, const CipherP& x0, int64_t k) {
  const CipherP x = ev_materialize(c, x0);
  CipherP r = new_cipher(c, x->v.n, x->v.level, x->v.t_exp);
  op_mul_scalar(c, x->v, k, r->v);
  r->v.nz = nz_scalar(x->v.nz, centered(k, c->tpow[x->v.t_exp]));
  return r;
}

static CipherP ev_const(bgv_ctx* c, const CipherP& x0, int64_t k) {
  const CipherP x = ev_materialize(c, x0);
  CipherP r = new_cipher(c, x->v.n, x->v.level, x->v.t_exp);
  op_add_const(c, x->v, k, r->v);
  r->v.nz = nz_add_const(x->v.nz, centered(k, c->tpow[x->v.t_exp]));
  return r;
}

static CipherP ev_neg(bgv_ctx* c, const CipherP& x0) {
  const CipherP x = ev_materialize(c, x0);
  CipherP r = new_cipher(c, x->v.n, x->v.level, x->v.t_exp);
  op_negate(c, x->v, r->v);
  r->v.nz = x->v.nz;
  return r;
}

// x^i by the power rule: h = 2^floor(log2 i); x^i = x^(i/2) x^(i/2) if i = h, else x^h x^(i-h).
static const CipherP& power(bgv_ctx* c, const bgv_keys* k, std::map<int, CipherP>& tab, int i) {
  auto it = tab.find(i);
  if (it != tab.end()) return it->second;
  int h = 1;
  while (2 * h <= i) h *= 2;
  CipherP r;
  if (i == h) {
    const CipherP& half = power(c, k, tab, i / 2);
    r = ev_mul(c, k, half, half);
  } else {
    const CipherP& a = power(c, k, tab, h);
    const CipherP& b = power(c, k, tab, i - h);
    r = ev_mul(c, k, a, b);
  }
  return tab[i] = r;
}

int eval_depth(int degree) {
  int k = 1;
  while (2 * k * k < degree + 1) k *= 2;
  int g = (degree + k) / k;
  int lk2 = 0;
  while ((1 << lk2) < k) ++lk2;
  int lg = 0;
  while ((1 << lg) < g - 1) ++lg;  // depth of y^(g-1) above y
  return lk2 + (g > 1 ? lg : 0) + 1;
}

// Device table [D+1][L] of the coefficients, each lifted to the centered range mod
// t and reduced mod every q_i; built once per (t_exp, coefficients) and kept.
static const double* coeff_table(bgv_ctx* c, int t_exp, const std::vector<int64_t>& cf) {
  auto key = std::make_pair(t_exp, cf);
  auto it = c->coeff_tabs.find(key);
  if (it != c->coeff_tabs.end()) return it->second;
  const int L = c->prm.L;
  const int64_t t = c->tpow[t_exp];
  // [rows][L] residues of the centered coefficients, then the centered values themselves
  std::vector<double> h(cf.size() * (size_t)L + cf.size());
  for (size_t r = 0; r < cf.size(); ++r) {
    scalar_table(c, centered(cf[r], t), L, &h[r * L]);
    h[cf.size() * (size_t)L + r] = (double)centered(cf[r], t);
  }
  double* d = nullptr;
  check_hip(c, hipMalloc((void**)&d, h.size() * sizeof(double)), "coefficient table");
  check_hip(c, hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice), "coefficient table");
  c->coeff_tabs[key] = d;
  return d;
}

// Baby-step/giant-step evaluation (Paterson-Stockmeyer, Theorem 2) with the
// schedule: k = smallest power of two with 2k^2 >= D+1 (k^2 >= D+1 for an
// odd-structured polynomial, see below), g = ceil((D+1)/k);
// baby powers x^2..x^k and giant powers y^2..y^(g-1) (y = x^k) by the power
// rule (the baby powers other than powers of two after the giants, each at the level its
// consumers need); inner sums over the nonzero coefficients with every power first brought
// to the level where the outer products meet (or its own lowest level if lower),
// scalar terms accumulated in increasing order and the constant added last; the
// outer products I_j y^j (j = 1..g-1, I_j not a constant) tensored at their lowest
// common level, summed, relinearised once and switched down one prime; then the
// scalar multiples c_jk y^j of constant inner sums in increasing j, then I_0.
// Every other product lowers its operands, relinearises and switches down one prime.
// The basic schedule (BGV_SCHED_BASIC) takes the dense split for every polynomial,
// forms each inner sum at the lowest level among its powers, and adds the outer terms
// in increasing j, each I_j y^j as one such product; then I_0.
CipherP ev_eval_poly(bgv_ctx* c, const bgv_keys* k, const CipherP& x, const std::vector<int64_t>& coeffs,
                     std::vector<CipherP>* giant_out, int* giant_k) {
  const int64_t t = c->tpow[x->v.t_exp];
  std::vector<int64_t> cf(coeffs.size());
  for (size_t i = 0; i < coeffs.size(); ++i) cf[i] = ((coeffs[i] % t) + t) % t;
  int D = (int)cf.size() - 1;
  while (D > 0 && cf[D] == 0) --D;
  if (D < 1) throw OpError{BGV_E_ARG};
  // An odd-structured polynomial (every even coefficient strictly between the
  // constant and the leading term zero: G_{p,e} for odd p, F_LT) needs only the odd
  // baby powers, so its split moves to k = smallest power of two with k^2 >= D+1.
  // The basic schedule keeps the dense split, own-level inner sums and one product
  // per outer term.
  const bool basic = c->schedule == BGV_SCHED_BASIC;
  bool odd = !basic && D >= 3;
  for (int i = 2; i < D && odd; i += 2)
    if (cf[i] != 0) odd = false;
  int kk = 1;
  while ((odd ? 1 : 2) * kk * kk < D + 1) kk *= 2;
  const int g = (D + kk) / kk;
  auto coef = [&](int n) -> int64_t { return n <= D ? cf[n] : 0; };
  c->stats.max_baby_k = std::max(c->stats.max_baby_k, kk);
  if (odd) c->stats.odd_splits += 1;

  const double* tab = coeff_table(c, x->v.t_exp, cf);
  // the centered coefficients follow the residue rows; they serve the exact split
  // accumulation of the inner sums when |c| <= (t - 1) / 2 < 2^24
  const double* scs = t <= ((int64_t)1 << 25) ? tab + cf.size() * (size_t)c->prm.L : nullptr;
  // Only the powers some term uses (and the factors the power rule builds them
  // from) are computed; each of them is the same product chain as in the full
  // table, so skipping the unused ones leaves every output word unchanged.
  std::vector<char> need_b(kk + 1, 0), need_g(std::max(g, 2), 0);
  need_b[kk] = 1;
  for (int j = 0; j < g; ++j) {
    bool any = false;
    for (int i = 1; i < kk; ++i)
      if (coef(j * kk + i) != 0) {
        need_b[i] = 1;
        any = true;
      }
    if (j >= 1 && (any || coef(j * kk) != 0)) need_g[j] = 1;
  }
  auto close = [](std::vector<char>& need) {
    for (int i = (int)need.size() - 1; i >= 2; --i) {
      if (!need[i]) continue;
      int h = 1;
      while (2 * h <= i) h *= 2;
      if (i == h) need[i / 2] = 1;
      else need[h] = need[i - h] = 1;
    }
  };
  close(need_b);
  close(need_g);
  SwitchedForms switched;  // operands switched down once for several lowerings
  std::map<int, CipherP> baby;
  baby[1] = x;
  // basic: every needed baby power by the power rule; fast: the powers of two up to x^k
  // here, the others after the giants
  for (int i = 2; i <= kk; ++i)
    if (need_b[i] && (basic || (i & (i - 1)) == 0)) power(c, k, baby, i);
  std::map<int, CipherP> giant;
  giant[1] = baby[kk];
  for (int j = 2; j < g; ++j)
    if (need_g[j]) power(c, k, giant, j);
  if (!basic) {
    // Each other needed baby power x^i = x^h x^(i-h) at the level its consumers need: F (the
    // lowest level among the giants of the non-constant inner sums, where the outer products
    // meet) for the inner sums, and one level above each power it is the second operand of.
    // It is formed by a product one level above that (lower if an operand is lower), its
    // operands brought down first; with no outer product, by the power rule as it comes.
    std::vector<int> late;
    for (int i = 3; i < kk; ++i)
      if (need_b[i] && (i & (i - 1)) != 0) late.push_back(i);
    int F = 1 << 30;
    for (int j = 1; j < g; ++j)
      for (int i = 1; i < kk; ++i)
        if (coef(j * kk + i) != 0) {
          F = std::min(F, giant[j]->v.level);
          break;
        }
    auto top_pow2 = [](int i) {
      int h = 1;
      while (2 * h <= i) h *= 2;
      return h;
    };
    if (F == 1 << 30) {
      for (int i : late) power(c, k, baby, i);
    } else {
      std::map<int, int> want;
      for (int i : late) want[i] = F;
      for (auto it = late.rbegin(); it != late.rend(); ++it) {
        auto w = want.find(*it - top_pow2(*it));
        if (w != want.end()) w->second = std::max(w->second, want[*it] + 1);
      }
      for (int i : late) {
        const int h = top_pow2(i);
        const CipherP a = baby[h], b = baby[i - h];
        const int lv = std::min(want[i] + 1, std::min(a->v.level, b->v.level));
        baby[i] = ev_mul(c, k, ev_lower_shared(c, a, lv, switched), ev_lower_shared(c, b, lv, switched));
      }
    }
  }

  std::map<std::pair<int, int>, CipherP> aligned;
  auto aligned_power = [&](int i, int lv) -> CipherP {
    auto key = std::make_pair(i, lv);
    auto it = aligned.find(key);
    if (it != aligned.end()) return it->second;
    CipherP r = ev_lower_shared(c, baby[i], lv, switched);
    aligned[key] = r;
    return r;
  };
  // an inner sum's estimate: its scalar terms accumulated in increasing i, then the constant
  const int64_t tt = c->tpow[x->v.t_exp];
  auto inner_nz = [&](int j, int lv, const std::vector<int>& terms_used) {
    int nz = 0;
    bool first = true;
    for (int i : terms_used) {
      const int tz = nz_scalar(aligned_power(i, lv)->v.nz, centered(coef(j * kk + i), tt));
      nz = first ? tz : nz_add(nz, tz);
      first = false;
    }
    if (coef(j * kk) != 0) nz = nz_add_const(nz, centered(coef(j * kk), tt));
    return nz;
  };

  struct Inner {
    bool is_const;
    int64_t cst;
    CipherP ct;
  };
  std::vector<Inner> inner(g);
  // Sums at the same level read the same aligned baby powers: one multi-output
  // pass per level reads each power once for all of them (a power absent from
  // a sum has no term there, so every sum gets the words of its own pass).
  // Every inner sum is formed at the level where the outer products meet (the lowest
  // level among the non-constant I_j and their y^j), or at its own lowest level if lower.
  std::map<int, std::vector<int>> by_level;
  std::vector<std::vector<int>> used(g);
  std::vector<int> own(g, 1 << 30);
  int meet = 1 << 30;
  for (int j = 0; j < g; ++j) {
    for (int i = 1; i < kk; ++i)
      if (coef(j * kk + i) != 0) {
        used[j].push_back(i);
        own[j] = std::min(own[j], baby[i]->v.level);
      }
    if (!basic && j >= 1 && !used[j].empty()) meet = std::min(meet, std::min(own[j], giant[j]->v.level));
  }
  for (int j = 0; j < g; ++j) {
    if (used[j].empty()) {
      inner[j] = Inner{true, coef(j * kk), nullptr};
      continue;
    }
    by_level[std::min(own[j], meet)].push_back(j);
  }
  for (auto& kv : by_level) {
    const int lv = kv.first;
    const std::vector<int>& js = kv.second;
    std::vector<int> terms;
    for (int j : js) terms.insert(terms.end(), used[j].begin(), used[j].end());
    std::sort(terms.begin(), terms.end());
    terms.erase(std::unique(terms.begin(), terms.end()), terms.end());
    if ((int)terms.size() <= lk::LC_MAXT) {
      std::vector<CipherP> keep;
      lk::LinMulti m{};
      for (size_t t = 0; t < terms.size(); ++t) {
        keep.push_back(aligned_power(terms[t], lv));
        m.x[t] = keep.back()->v.d;
        m.xs[t] = lstride(keep.back()->v);
      }
      for (size_t s0 = 0; s0 < js.size(); s0 += lk::LC_MAXO) {
        const int no = (int)std::min<size_t>(lk::LC_MAXO, js.size() - s0);
        for (int o = 0; o < no; ++o) {
          const int j = js[s0 + o];
          CipherP acc = new_cipher(c, x->v.n, lv, x->v.t_exp);
          m.out[o] = acc->v.d;
          for (size_t t = 0; t < terms.size(); ++t)
            m.row[o][t] = coef(j * kk + terms[t]) != 0 ? j * kk + terms[t] : -1;
          m.cst_row[o] = coef(j * kk) != 0 ? j * kk : -1;
          acc->v.nz = inner_nz(j, lv, used[j]);
          inner[j] = Inner{false, 0, acc};
        }
        c->stats.max_inner_terms = std::max(c->stats.max_inner_terms, (int)terms.size());
        c->stats.max_inner_outputs = std::max(c->stats.max_inner_outputs, no);
        algo(c, 2.0 * lv * (terms.size() + no) * x->v.n);
        lk::lincomb_multi(c, m, (int)terms.size(), no, tab, c->prm.L, scs, x->v.n, lv);
      }
      continue;
    }
    for (int j : js) {
      // sum_i c_{jk+i} x^i (+ c_{jk}) in passes of at most 16 terms: the scalar
      // products and additions are exact in every Z_q_i, so the linear
      // combinations give the same words as the term-by-term accumulation
      const int64_t cst = coef(j * kk);
      std::vector<CipherP> keep;
      std::vector<const uint64_t*> xs;
      std::vector<int> rws;
      for (int i : used[j]) {
        keep.push_back(ev_materialize(c, aligned_power(i, lv)));  // the single-sum kernel reads no views
        xs.push_back(keep.back()->v.d);
        rws.push_back(j * kk + i);
      }
      CipherP acc = new_cipher(c, x->v.n, lv, x->v.t_exp);
      for (size_t s = 0; s < xs.size(); s += 16) {
        const int nt = (int)std::min<size_t>(16, xs.size() - s);
        CipherP part = s == 0 ? acc : new_cipher(c, x->v.n, lv, x->v.t_exp);
        algo(c, 2.0 * lv * (nt + 1) * x->v.n);
        lk::lincomb(c, xs.data() + s, rws.data() + s, nt, tab, c->prm.L, (s == 0 && cst != 0) ? j * kk : -1,
                    part->v.d, x->v.n, lv);
        if (s > 0) op_add_sub(c, acc->v, part->v, acc->v, 0);
      }
      acc->v.nz = inner_nz(j, lv, used[j]);
      inner[j] = Inner{false, 0, acc};
    }
  }
  // the inner sums hold everything the outer sum needs from the baby steps (the switched
  // forms are keyed by their sources' addresses: dropped before any source is)
  aligned.clear();
  switched.clear();
  for (auto it = baby.begin(); it != baby.end();) it = (it->first != 1 && it->first != kk) ? baby.erase(it) : std::next(it);
  // outer sum: the products I_j y^j (relinearised once together in the fast schedule),
  // the scalar multiples c_jk y^j of constant inner sums, then I_0
  CipherP result;
  if (basic) {
    // in increasing j: I_j y^j as one product, or c_jk y^j, added at the lower level
    for (int j = 1; j < g; ++j) {
      CipherP term;
      if (!inner[j].is_const) term = ev_mul(c, k, inner[j].ct, giant[j]);
      else if (inner[j].cst != 0) term = ev_scalar(c, giant[j], inner[j].cst);
      else continue;
      result = result ? ev_add(c, result, term) : term;
    }
  } else {
    // the products I_j y^j relinearised once together; the scalar multiples c_jk y^j of
    // constant inner sums (increasing j), then I_0, join them before the switch when they are
    // at that level or above, otherwise they are added after it
    std::vector<std::pair<CipherP, CipherP>> pairs;
    for (int j = 1; j < g; ++j)
      if (!inner[j].is_const) pairs.push_back({inner[j].ct, giant[j]});
    std::vector<int> late_scalars;
    if (!pairs.empty()) {
      const int lv = lazy_level(pairs);
      std::vector<std::pair<int64_t, CipherP>> addends;
      for (int j = 1; j < g; ++j) {
        if (!inner[j].is_const || inner[j].cst == 0) continue;
        if (giant[j]->v.level >= lv) addends.push_back({inner[j].cst, giant[j]});
        else late_scalars.push_back(j);
      }
      if (!inner[0].is_const && inner[0].ct->v.level >= lv) {
        addends.push_back({1, inner[0].ct});
        inner[0].ct = nullptr;  // folded
      }
      result = ev_lazy_products(c, k, pairs, addends);
    } else {
      for (int j = 1; j < g; ++j)
        if (inner[j].is_const && inner[j].cst != 0) late_scalars.push_back(j);
    }
    pairs.clear();
    for (int j : late_scalars) {
      CipherP term = ev_scalar(c, giant[j], inner[j].cst);
      result = result ? ev_add(c, result, term) : term;
    }
  }
  if (inner[0].is_const) {
    if (!result) throw OpError{BGV_E_ARG};
    if (inner[0].cst != 0) result = ev_const(c, result, inner[0].cst);
  } else if (inner[0].ct) {
    result = result ? ev_add(c, result, inner[0].ct) : inner[0].ct;
  }
  if (giant_out) {
    giant_out->assign(g, nullptr);
    for (int j = 1; j < g; ++j)
      if (giant.count(j)) (*giant_out)[j] = giant[j];
    *giant_k = kk;
  }
  return result;
}

// Algorithm 3: the balanced base-p digits of a value tagged t = p^e, least significant
// first.  G_{p,e'} of the current value b (tagged p^e') is its lowest digit (Lemma 3);
// b minus that digit is a multiple of p, and DivideByP of it is the value of the remaining
// digits, tagged p^(e'-1).  A value tagged p is the top digit.  Digits are tagged t = p.
std::vector<CipherP> ev_space_reduce(bgv_ctx* c, const bgv_keys* k, const CipherP& x) {
  const int e = x->v.t_exp;
  if (e == 1) return {x};
  if (e >= (int)c->gpe.size() || c->gpe[e].empty()) throw OpError{BGV_E_UNSUPPORTED};
  std::vector<CipherP> digits;
  CipherP b = x;
  for (int i = 0; i < e - 1; ++i) {
    const int te = e - i;  // b is tagged t = p^te
    CipherP ai = ev_eval_poly(c, k, b, c->gpe[te]);
    CipherP bb = ev_lower(c, b, ai->v.level);
    CipherP d = new_cipher(c, x->v.n, ai->v.level, te);
    op_add_sub(c, bb->v, ai->v, d->v, 1);
    d->v.nz = nz_add(bb->v.nz, ai->v.nz);
    CipherP nb = new_cipher(c, x->v.n, ai->v.level, te - 1);
    op_divide_by_p(c, d->v, nb->v);
    nb->v.nz = nz_divide_by_p(c, d->v.nz);
    digits.push_back(with_t(ai, 1));
    b = nb;
  }
  digits.push_back(b);
  return digits;
}

static CipherP one_minus(bgv_ctx* c, const CipherP& x) { return ev_const(c, ev_neg(c, x), 1); }

// Algorithm 4 (digits least significant first).  A value is below zero exactly when its
// most significant nonzero balanced digit is: a fold from the top digit down carries
// (lt, eq) -- the digits read so far are below zero / all zero -- and absorbs digit i as
// (lt + eq LT_i, eq EQ_i); the last digit's eq is never formed.
CipherP ev_compare(bgv_ctx* c, const bgv_keys* k, const std::vector<CipherP>& digits, int op) {
  const int top = (int)digits.size() - 1;
  const int p = c->prm.p;
  auto eq_digit = [&](const CipherP& x) {
    std::map<int, CipherP> tab;
    tab[1] = x;
    return one_minus(c, power(c, k, tab, p - 1));
  };
  if (op == BGV_OP_LE || op == BGV_OP_GE || op == BGV_OP_NEQ) {
    const int base = op == BGV_OP_LE ? BGV_OP_GT : (op == BGV_OP_GE ? BGV_OP_LT : BGV_OP_EQ);
    return one_minus(c, ev_compare(c, k, digits, base));  // 1 - base
  }
  if (op == BGV_OP_EQ) {
    CipherP eq = eq_digit(digits[top]);
    for (int i = top - 1; i >= 0; --i) eq = ev_mul(c, k, eq, eq_digit(digits[i]));
    return eq;
  }
  const std::vector<int64_t>& fdig = op == BGV_OP_GT ? c->fgt : c->flt;
  std::vector<CipherP> giants;
  int kk = 0;
  CipherP lt = ev_eval_poly(c, k, digits[top], fdig, &giants, &kk);
  CipherP eq;
  if (top > 0) {
    // x^(p-1) is the last giant power when (g-1) k = p-1 (same products as the power rule)
    const int g = (int)giants.size();
    if (g > 1 && (g - 1) * kk == p - 1 && giants[g - 1]) eq = one_minus(c, giants[g - 1]);
    else eq = eq_digit(digits[top]);
  }
  giants.clear();
  for (int i = top - 1; i >= 0; --i) {
    lt = ev_add(c, lt, ev_mul(c, k, eq, ev_eval_poly(c, k, digits[i], fdig)));
    if (i > 0) eq = ev_mul(c, k, eq, eq_digit(digits[i]));
  }
  return lt;
}

CipherP ev_space_raise(bgv_ctx* c, const bgv_keys* k, const CipherP& x) {
  const int r = c->prm.r;
  if (r == 1) return with_t(x, 1);
  if (r >= (int)c->gpe.size() || c->gpe[r].empty()) throw OpError{BGV_E_UNSUPPORTED};
  return ev_eval_poly(c, k, with_t(x, r), c->gpe[r]);
}

CipherP ev_rotate_sum(bgv_ctx* c, const bgv_keys* k, const CipherP& x) {
  CipherP acc = ev_materialize(c, x);
  for (int i = 1; i < c->ell / 2; i *= 2) {
    CipherP r = new_cipher(c, acc->v.n, acc->v.level, acc->v.t_exp);
    op_rotate(c, k, acc->v, galois_elt(c, i), r->v);
    r->v.nz = nz_key_switch(c, acc->v.nz, acc->v.t_exp, acc->v.level);
    acc = ev_add(c, acc, r);
  }
  CipherP r = new_cipher(c, acc->v.n, acc->v.level, acc->v.t_exp);
  op_rotate(c, k, acc->v, galois_elt(c, BGV_ROW_SWAP), r->v);
  r->v.nz = nz_key_switch(c, acc->v.nz, acc->v.t_exp, acc->v.level);
  return ev_add(c, acc, r);
}

// [x < y] in the number space: reduce -> compare -> raise of x - y (of x alone if y is null)
CipherP ev_less_than(bgv_ctx* c, const bgv_keys* k, const CipherP& x, const CipherP& y) {
  CipherP d = x;
  if (y) {
    // y is a batch of the same size or one ciphertext broadcast over x
    if (y->v.n != x->v.n && y->v.n != 1) throw OpError{BGV_E_ARG};
    d = new_cipher(c, x->v.n, x->v.level, x->v.t_exp);
    op_add_sub(c, x->v, y->v, d->v, 1);
    d->v.nz = nz_add(x->v.nz, y->v.nz);
  }
  std::vector<CipherP> dg = ev_space_reduce(c, k, d);
  return ev_space_raise(c, k, ev_compare(c, k, dg, BGV_OP_LT));
}

// the ciphertexts of a batch summed; the estimate bounds the n terms by the largest
// (a + lgc(n)) rather than chaining n - 1 pairwise sums
CipherP ev_batch_sum(bgv_ctx* c, const CipherP& x0) {
  const CipherP x = ev_materialize(c, x0);
  algo(c, 2.0 * x->v.level * (x->v.n + 1));
  CipherP r = new_cipher(c, 1, x->v.level, x->v.t_exp);
  lk::batch_sum(c, x->v.d, r->v.d, x->v.n, x->v.level);
  r->v.nz = nz_sum_of(x->v.nz, x->v.n);
  return r;
}

// b * c formed where it is consumed: by a product one level above `level` (the level of
// the factor it meets; lower if an operand is lower), its operands brought down first.  In
// the basic schedule, at the operands' own level.
static CipherP ev_product_at(bgv_ctx* c, const bgv_keys* k, const CipherP& b, const CipherP& cc, int level) {
  if (c->schedule == BGV_SCHED_BASIC) return ev_mul(c, k, b, cc);
  const int lv = std::min(level + 1, std::min(b->v.level, cc->v.level));
  return ev_mul(c, k, ev_lower(c, b, lv), ev_lower(c, cc, lv));
}

// SUM(b*c WHERE a < thr): [a < thr] * (b * c) per ciphertext (b * c formed at the
// predicate's level), summed over the batch, then rotate-and-sum over the slots.
CipherP ev_filter_products(bgv_ctx* c, const bgv_keys* k, const CipherP& a, const CipherP& thr, const CipherP& b,
                           const CipherP& cc) {
  CipherP lt = ev_less_than(c, k, a, thr);
  return ev_mul(c, k, lt, ev_product_at(c, k, b, cc, lt->v.level));
}

CipherP ev_filter_sum(bgv_ctx* c, const bgv_keys* k, const CipherP& a, const CipherP& thr, const CipherP& b,
                      const CipherP& cc) {
  return ev_rotate_sum(c, k, ev_batch_sum(c, ev_filter_products(c, k, a, thr, b, cc)));
}

// [every predicate holds] * (b * c) per ciphertext.  Predicate i compares column i with
// threshold i: op_i applied to the digits of col_i - thr_i (reduce, then compare; the results
// are 0/1 tagged t = p).  The conjunction is the product of those results in the digit space,
// formed as a balanced tree over the predicates in their order (pairs (0,1), (2,3), .., then
// pairs of those), raised once to t = p^r and multiplied by b * c, formed at that level.
CipherP ev_filter_and_products(bgv_ctx* c, const bgv_keys* k, const std::vector<CipherP>& cols,
                               const std::vector<CipherP>& thrs, const std::vector<int>& ops, const CipherP& b,
                               const CipherP& cc) {
  std::vector<CipherP> preds;
  for (size_t i = 0; i < cols.size(); ++i) {
    const CipherP& x = cols[i];
    const CipherP& y = thrs[i];
    if (y->v.n != x->v.n && y->v.n != 1) throw OpError{BGV_E_ARG};
    CipherP d = new_cipher(c, x->v.n, x->v.level, x->v.t_exp);
    op_add_sub(c, x->v, y->v, d->v, 1);
    d->v.nz = nz_add(x->v.nz, y->v.nz);
    preds.push_back(ev_compare(c, k, ev_space_reduce(c, k, d), ops[i]));
  }
  while (preds.size() > 1) {
    std::vector<CipherP> next;
    for (size_t i = 0; i + 1 < preds.size(); i += 2) next.push_back(ev_mul(c, k, preds[i], preds[i + 1]));
    if (preds.size() % 2) next.push_back(preds.back());
    preds.swap(next);
  }
  CipherP m = ev_space_raise(c, k, preds[0]);
  return ev_mul(c, k, m, ev_product_at(c, k, b, cc, m->v.level));
}

CipherP ev_filter_and_sum(bgv_ctx* c, const bgv_keys* k, const std::vector<CipherP>& cols,
                          const std::vector<CipherP>& thrs, const std::vector<int>& ops, const CipherP& b,
                          const CipherP& cc) {
  return ev_rotate_sum(c, k, ev_batch_sum(c, ev_filter_and_products(c, k, cols, thrs, ops, b, cc)));
}

CipherP ev_relu(bgv_ctx* c, const bgv_keys* k, const CipherP& x) {
  CipherP lt = ev_less_than(c, k, x, nullptr);
  return ev_mul(c, k, x, ev_const(c, ev_neg(c, lt), 1));
}
