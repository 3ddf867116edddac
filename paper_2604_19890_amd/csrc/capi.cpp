// extern "C" entry points: argument validation, then the operation layer.
// Every check that can fail runs on the host before any work is enqueued.
#include <algorithm>
#include <cstring>
#include <new>

#include "host_nt.hpp"
#include "ops.hpp"

#define BGV_EXPORT extern "C" __attribute__((visibility("default")))

namespace {

bgv_status fail(bgv_ctx* c, bgv_status st, const char* msg) {
  if (c && msg) c->err = msg;
  return st;
}

bgv_status check_in(bgv_ctx* c, const bgv_ct* x, const char* name) {
  if (!x || !x->d) return fail(c, BGV_E_ARG, name);
  if (x->n < 1) return fail(c, BGV_E_ARG, "batch count must be >= 1");
  if (x->n > c->max_batch()) return fail(c, BGV_E_ARG, "batch count above the context's max_batch");
  if (x->level < 1 || x->level > c->prm.L) return fail(c, BGV_E_LEVEL, "level out of range");
  if (x->t_exp < 1 || x->t_exp > c->prm.r) return fail(c, BGV_E_PTXT_MOD, "t_exp out of range");
  if (x->cap_words < (int64_t)x->n * (int64_t)ct_words(c, x->level)) return fail(c, BGV_E_ARG, "input buffer too small");
  return BGV_OK;
}

bgv_status check_out(bgv_ctx* c, bgv_ct* out, int n, int level) {
  if (!out || !out->d) return fail(c, BGV_E_ARG, "null output");
  if (out->cap_words < (int64_t)n * (int64_t)ct_words(c, level)) return fail(c, BGV_E_ARG, "output buffer too small");
  return BGV_OK;
}

CtV view(const bgv_ct* x) {
  CtV v;
  v.d = x->d;
  v.n = x->n;
  v.level = x->level;
  v.t_exp = x->t_exp;
  v.nz = x->noise > 0 ? x->noise : 0;
  return v;
}

void set_out(bgv_ct* out, int n, int level, int t_exp, int nz) {
  out->n = n;
  out->level = level;
  out->t_exp = t_exp;
  out->noise = nz;
}

CipherP borrow(const bgv_ct* x) {
  auto p = std::make_shared<Cipher>();
  p->v = view(x);
  return p;
}

// write an owned result into a caller batch
bgv_status deliver(bgv_ctx* c, const CipherP& r, bgv_ct* out) {
  bgv_status st = check_out(c, out, r->v.n, r->v.level);
  if (st != BGV_OK) return st;
  const CipherP flat = ev_materialize(c, r);  // a view of a deeper batch's lower limbs is copied first
  CtV o = flat->v;
  o.d = out->d;
  op_copy(c, flat->v, o);
  set_out(out, r->v.n, r->v.level, r->v.t_exp, r->v.nz);
  return BGV_OK;
}

template <class F>
bgv_status guarded(bgv_ctx* c, F f) {
  try {
    return f();
  } catch (const OpError& e) {
    if (c && c->err.empty()) c->err = "operation failed";
    return e.st;
  } catch (const std::bad_alloc&) {
    return fail(c, BGV_E_OOM, "host allocation failed");
  }
}

#define CHECK(x)                     \
  do {                               \
    bgv_status _s = (x);             \
    if (_s != BGV_OK) return _s;     \
  } while (0)

#define NEED_CTX(c) \
  if (!(c)) return BGV_E_ARG;  \
  (c)->err.clear();

}  // namespace

BGV_EXPORT bgv_status bgv_ctx_create(const bgv_params* prm, void* stream, bgv_ctx** out) {
  if (!prm || !out) return BGV_E_ARG;
  bgv_ctx* c = new (std::nothrow) bgv_ctx();
  if (!c) return BGV_E_OOM;
  bgv_status st;
  try {
    st = ctx_build(c, prm, (hipStream_t)stream);
  } catch (const std::bad_alloc&) {
    st = BGV_E_OOM;
  }
  if (st != BGV_OK) {
    *out = c;  // lets the caller read bgv_last_error; bgv_ctx_destroy frees it
    return st;
  }
  *out = c;
  return BGV_OK;
}

BGV_EXPORT void bgv_ctx_destroy(bgv_ctx* c) {
  if (!c) return;
  ctx_free(c);
  delete c;
}

BGV_EXPORT bgv_status bgv_set_stream(bgv_ctx* c, void* stream) {
  NEED_CTX(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  c->stream = (hipStream_t)stream;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_ctx_info(const bgv_ctx* c, bgv_info* o) {
  if (!c || !o) return BGV_E_ARG;
  o->N = c->N;
  o->log_n = c->logN;
  o->p = c->prm.p;
  o->r = c->prm.r;
  o->L = c->prm.L;
  o->K = c->prm.K;
  o->alpha = c->alpha;
  o->dnum = c->dnum;
  o->slots = c->ell;
  o->d = c->dslot;
  o->t = c->t_full;
  o->max_batch = c->max_batch();
  o->_pad = 0;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_ctx_primes(const bgv_ctx* c, uint64_t* out) {
  if (!c || !out) return BGV_E_ARG;
  std::memcpy(out, c->primes.data(), c->primes.size() * sizeof(uint64_t));
  return BGV_OK;
}

BGV_EXPORT int64_t bgv_ct_words(const bgv_ctx* c, int32_t level) {
  if (!c || level < 1) return 0;
  return (int64_t)ct_words(c, level);
}

BGV_EXPORT bgv_status bgv_sync(bgv_ctx* c) {
  NEED_CTX(c);
  hipError_t e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) {
    c->err = std::string("device error: ") + hipGetErrorString(e);
    return BGV_E_DEVICE;
  }
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_set_modup_fused(bgv_ctx* c, int32_t on) {
  NEED_CTX(c);
  if (on != 0 && on != 1) return fail(c, BGV_E_ARG, "0 or 1");
  c->modup_fused = on;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_set_moddown_fused(bgv_ctx* c, int32_t on) {
  NEED_CTX(c);
  if (on < 0 || on > 2) return fail(c, BGV_E_ARG, "0, 1 or 2");
  c->moddown_fused = on;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_set_ntt_coop(bgv_ctx* c, int32_t mode, int32_t lookahead) {
  NEED_CTX(c);
  if (mode < 0 || mode > 1 || lookahead < 0 || lookahead > 16) return fail(c, BGV_E_ARG, "mode 0/1, lookahead 0..16");
  if (mode == 1) return fail(c, BGV_E_UNSUPPORTED, "the XCD-local transform is switched off");
  return BGV_OK;
}

BGV_EXPORT const char* bgv_last_error(const bgv_ctx* c) { return c ? c->err.c_str() : "null context"; }

BGV_EXPORT bgv_status bgv_keygen(bgv_ctx* c, const int8_t* s, const uint64_t* a, const int32_t* e,
                                 const int32_t* steps, int32_t n_steps, int32_t with_conj, bgv_keys** out) {
  NEED_CTX(c);
  if (!s || !a || !e || !out || n_steps < 0 || (n_steps > 0 && !steps)) return fail(c, BGV_E_ARG, "bad keygen arguments");
  std::vector<int> gal;
  for (int i = 0; i < n_steps; ++i) gal.push_back(galois_elt(c, steps[i]));
  if (with_conj) gal.push_back(galois_elt(c, BGV_ROW_SWAP));
  bgv_keys* k = new (std::nothrow) bgv_keys();
  if (!k) return BGV_E_OOM;
  k->ctx = c;
  bgv_status st = guarded(c, [&] { return op_keygen(c, s, a, e, gal, k); });
  if (st != BGV_OK) {
    bgv_keys_destroy(k);
    return st;
  }
  *out = k;
  return BGV_OK;
}

BGV_EXPORT void bgv_keys_destroy(bgv_keys* k) {
  if (!k) return;
  if (k->ctx && k->ctx->stream) (void)hipStreamSynchronize(k->ctx->stream);
  if (k->relin) (void)hipFree(k->relin);
  for (auto& kv : k->galois) (void)hipFree(kv.second);
  delete k;
}

BGV_EXPORT int64_t bgv_keys_bytes(const bgv_keys* k) { return k ? k->bytes : 0; }

BGV_EXPORT bgv_status bgv_encrypt(bgv_ctx* c, const int8_t* s, const uint64_t* slots, const uint64_t* c1,
                                  const int32_t* e, bgv_ct* out) {
  NEED_CTX(c);
  if (!s || !slots || !c1 || !e || !out || out->n < 1) return fail(c, BGV_E_ARG, "bad encrypt arguments");
  if (out->n > c->max_batch()) return fail(c, BGV_E_ARG, "batch count above the context's max_batch");
  CHECK(check_out(c, out, out->n, c->prm.L));
  set_out(out, out->n, c->prm.L, c->prm.r, c->nzm.fresh);
  return guarded(c, [&] { return op_encrypt(c, s, slots, c1, e, view(out)); });
}

BGV_EXPORT bgv_status bgv_decrypt(bgv_ctx* c, const int8_t* s, const bgv_ct* in, uint64_t* slots, uint8_t* nonconst) {
  NEED_CTX(c);
  CHECK(check_in(c, in, "null input"));
  if (!s || !slots) return fail(c, BGV_E_ARG, "bad decrypt arguments");
  return guarded(c, [&] { return op_decrypt(c, s, view(in), slots, nonconst); });
}

static bgv_status binary_check(bgv_ctx* c, const bgv_ct* a, const bgv_ct* b) {
  CHECK(check_in(c, a, "null a"));
  CHECK(check_in(c, b, "null b"));
  if (a->level != b->level) return fail(c, BGV_E_LEVEL, "operands at different levels");
  if (a->t_exp != b->t_exp) return fail(c, BGV_E_PTXT_MOD, "operands with different plaintext moduli");
  if (b->n != a->n && b->n != 1) return fail(c, BGV_E_ARG, "batch sizes differ");
  return BGV_OK;
}

static bgv_status addsub(bgv_ctx* c, const bgv_ct* a, const bgv_ct* b, bgv_ct* out, int op) {
  NEED_CTX(c);
  CHECK(binary_check(c, a, b));
  CHECK(check_out(c, out, a->n, a->level));
  bgv_ct A = *a, B = *b;
  bgv_status st = guarded(c, [&] {
    CtV o = view(&A);
    o.d = out->d;
    op_add_sub(c, view(&A), view(&B), o, op);
    return BGV_OK;
  });
  if (st == BGV_OK) set_out(out, A.n, A.level, A.t_exp, nz_add(view(&A).nz, view(&B).nz));
  return st;
}

BGV_EXPORT bgv_status bgv_add(bgv_ctx* c, const bgv_ct* a, const bgv_ct* b, bgv_ct* out) { return addsub(c, a, b, out, 0); }
BGV_EXPORT bgv_status bgv_sub(bgv_ctx* c, const bgv_ct* a, const bgv_ct* b, bgv_ct* out) { return addsub(c, a, b, out, 1); }

template <class F>
static bgv_status unary(bgv_ctx* c, const bgv_ct* a, bgv_ct* out, int out_level, int out_t, int out_nz, F f) {
  NEED_CTX(c);
  CHECK(check_in(c, a, "null input"));
  CHECK(check_out(c, out, a->n, out_level));
  bgv_ct A = *a;
  bgv_status st = guarded(c, [&] {
    CtV o = view(&A);
    o.d = out->d;
    o.level = out_level;
    o.t_exp = out_t;
    f(view(&A), o);
    return BGV_OK;
  });
  if (st == BGV_OK) set_out(out, A.n, out_level, out_t, out_nz);
  return st;
}

BGV_EXPORT bgv_status bgv_negate(bgv_ctx* c, const bgv_ct* a, bgv_ct* out) {
  if (!a || !c) return BGV_E_ARG;
  return unary(c, a, out, a->level, a->t_exp, view(a).nz, [&](const CtV& x, const CtV& o) { op_negate(c, x, o); });
}

BGV_EXPORT bgv_status bgv_mul_scalar(bgv_ctx* c, const bgv_ct* a, int64_t k, bgv_ct* out) {
  if (!a || !c) return BGV_E_ARG;
  if (a->t_exp < 1 || a->t_exp > c->prm.r) return fail(c, BGV_E_PTXT_MOD, "t_exp out of range");
  const int nz = nz_scalar(view(a).nz, hnt::centered(k, c->tpow[a->t_exp]));
  return unary(c, a, out, a->level, a->t_exp, nz, [&](const CtV& x, const CtV& o) { op_mul_scalar(c, x, k, o); });
}

BGV_EXPORT bgv_status bgv_add_const(bgv_ctx* c, const bgv_ct* a, int64_t k, bgv_ct* out) {
  if (!a || !c) return BGV_E_ARG;
  if (a->t_exp < 1 || a->t_exp > c->prm.r) return fail(c, BGV_E_PTXT_MOD, "t_exp out of range");
  const int nz = nz_add_const(view(a).nz, hnt::centered(k, c->tpow[a->t_exp]));
  return unary(c, a, out, a->level, a->t_exp, nz, [&](const CtV& x, const CtV& o) { op_add_const(c, x, k, o); });
}

BGV_EXPORT bgv_status bgv_divide_by_p(bgv_ctx* c, const bgv_ct* a, bgv_ct* out) {
  if (!a || !c) return BGV_E_ARG;
  if (a->t_exp < 2) return fail(c, BGV_E_PTXT_MOD, "DivideByP needs t = p^k with k >= 2");
  return unary(c, a, out, a->level, a->t_exp - 1, nz_divide_by_p(c, view(a).nz),
               [&](const CtV& x, const CtV& o) { op_divide_by_p(c, x, o); });
}

BGV_EXPORT bgv_status bgv_set_t_exp(bgv_ctx* c, bgv_ct* ct, int32_t t_exp) {
  NEED_CTX(c);
  if (!ct) return BGV_E_ARG;
  if (t_exp < 1 || t_exp > c->prm.r) return fail(c, BGV_E_PTXT_MOD, "t_exp out of range");
  ct->t_exp = t_exp;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_mul_relin(bgv_ctx* c, const bgv_keys* k, const bgv_ct* a, const bgv_ct* b, bgv_ct* out) {
  NEED_CTX(c);
  if (!k || !k->relin) return fail(c, BGV_E_NOKEY, "no relinearisation key");
  CHECK(binary_check(c, a, b));
  CHECK(check_out(c, out, a->n, a->level));
  bgv_ct A = *a, B = *b;
  bgv_status st = guarded(c, [&] {
    CtV o = view(&A);
    o.d = out->d;
    op_mul_relin(c, k, view(&A), view(&B), o);
    return BGV_OK;
  });
  if (st == BGV_OK)
    set_out(out, A.n, A.level, A.t_exp,
            nz_key_switch(c, nz_tensor(c, view(&A).nz, view(&B).nz), A.t_exp, A.level));
  return st;
}

BGV_EXPORT bgv_status bgv_rotate(bgv_ctx* c, const bgv_keys* k, const bgv_ct* in, int32_t step, bgv_ct* out) {
  NEED_CTX(c);
  if (!k) return fail(c, BGV_E_NOKEY, "no keys");
  CHECK(check_in(c, in, "null input"));
  const int g = galois_elt(c, step);
  if (!k->galois.count(g)) return fail(c, BGV_E_NOKEY, "no Galois key for this rotation");
  return unary(c, in, out, in->level, in->t_exp, nz_key_switch(c, view(in).nz, in->t_exp, in->level),
               [&](const CtV& x, const CtV& o) { op_rotate(c, k, x, g, o); });
}

BGV_EXPORT bgv_status bgv_mod_switch(bgv_ctx* c, const bgv_ct* in, bgv_ct* out) {
  NEED_CTX(c);
  CHECK(check_in(c, in, "null input"));
  if (in->level < 2) return fail(c, BGV_E_LEVEL, "no prime left to drop");
  return unary(c, in, out, in->level - 1, in->t_exp, nz_switch(c, view(in).nz, in->t_exp),
               [&](const CtV& x, const CtV& o) { op_mod_switch(c, x, o); });
}

BGV_EXPORT bgv_status bgv_mod_switch_noalloc(bgv_ctx* c, const bgv_ct* in, bgv_ct* out) {
  NEED_CTX(c);
  CHECK(check_in(c, in, "null input"));
  if (in->level < 2) return fail(c, BGV_E_LEVEL, "no prime left to drop");
  if (!c->noalloc_scratch) return fail(c, BGV_E_DEVICE, "the allocation-free scratch is not available on this device");
  // T [n][2][N] and W [n][2][level-1][N]
  const int64_t t_words = (int64_t)in->n * 2 * c->N;
  const int64_t need = t_words + (int64_t)in->n * 2 * (in->level - 1) * c->N;
  if (need > BGV_NOALLOC_SCRATCH_WORDS)
    return fail(c, BGV_E_ARG, "the switch needs more scratch than the allocation-free variant holds");
  uint64_t* T = c->noalloc_scratch;
  uint64_t* W = T + t_words;
  return unary(c, in, out, in->level - 1, in->t_exp, nz_switch(c, view(in).nz, in->t_exp),
               [&](const CtV& x, const CtV& o) { op_mod_switch_with(c, x, o, T, W); });
}

BGV_EXPORT bgv_status bgv_mod_switch_to(bgv_ctx* c, const bgv_ct* in, int32_t level, bgv_ct* out) {
  NEED_CTX(c);
  CHECK(check_in(c, in, "null input"));
  if (level < 1 || level > in->level) return fail(c, BGV_E_LEVEL, "target level out of range");
  int nz = view(in).nz;
  for (int l = in->level; l > level; --l) nz = nz_switch(c, nz, in->t_exp);
  return unary(c, in, out, level, in->t_exp, nz, [&](const CtV& x, const CtV& o) { op_mod_switch_to(c, x, level, o); });
}

BGV_EXPORT bgv_status bgv_eval_poly(bgv_ctx* c, const bgv_keys* k, const bgv_ct* in, const int64_t* coeffs,
                                    int32_t degree, bgv_ct* out) {
  NEED_CTX(c);
  if (!k || !coeffs || degree < 1 || !out) return fail(c, BGV_E_ARG, "bad eval_poly arguments");
  CHECK(check_in(c, in, "null input"));
  std::vector<int64_t> cf(coeffs, coeffs + degree + 1);
  return guarded(c, [&] {
    CipherP r = ev_eval_poly(c, k, borrow(in), cf);
    return deliver(c, r, out);
  });
}

BGV_EXPORT bgv_status bgv_space_reduce(bgv_ctx* c, const bgv_keys* k, const bgv_ct* in, bgv_ct* digits) {
  NEED_CTX(c);
  if (!k || !digits) return fail(c, BGV_E_ARG, "bad space_reduce arguments");
  CHECK(check_in(c, in, "null input"));
  return guarded(c, [&] {
    std::vector<CipherP> d = ev_space_reduce(c, k, borrow(in));
    for (size_t i = 0; i < d.size(); ++i) CHECK(check_out(c, &digits[i], d[i]->v.n, d[i]->v.level));
    for (size_t i = 0; i < d.size(); ++i) CHECK(deliver(c, d[i], &digits[i]));
    return BGV_OK;
  });
}

BGV_EXPORT bgv_status bgv_compare(bgv_ctx* c, const bgv_keys* k, const bgv_ct* digits, int32_t r, int32_t op,
                                  bgv_ct* out) {
  NEED_CTX(c);
  if (!k || !digits || r < 1 || r > c->prm.r || op < BGV_OP_LT || op > BGV_OP_NEQ)
    return fail(c, BGV_E_ARG, "bad compare arguments");
  std::vector<CipherP> d;
  for (int i = 0; i < r; ++i) {
    CHECK(check_in(c, &digits[i], "null digit"));
    if (digits[i].t_exp != 1) return fail(c, BGV_E_PTXT_MOD, "digits must have t = p");
    if (digits[i].n != digits[0].n) return fail(c, BGV_E_ARG, "digit batches differ");
    d.push_back(borrow(&digits[i]));
  }
  return guarded(c, [&] { return deliver(c, ev_compare(c, k, d, op), out); });
}

BGV_EXPORT bgv_status bgv_space_raise(bgv_ctx* c, const bgv_keys* k, const bgv_ct* in, bgv_ct* out) {
  NEED_CTX(c);
  if (!k) return fail(c, BGV_E_ARG, "no keys");
  CHECK(check_in(c, in, "null input"));
  if (in->t_exp != 1) return fail(c, BGV_E_PTXT_MOD, "raising starts from t = p");
  return guarded(c, [&] { return deliver(c, ev_space_raise(c, k, borrow(in)), out); });
}

BGV_EXPORT bgv_status bgv_less_than(bgv_ctx* c, const bgv_keys* k, const bgv_ct* x, const bgv_ct* y, bgv_ct* out) {
  NEED_CTX(c);
  if (!k) return fail(c, BGV_E_ARG, "no keys");
  CHECK(check_in(c, x, "null x"));
  if (y) CHECK(binary_check(c, x, y));  // y: same batch size or a single broadcast ciphertext
  if (x->t_exp != c->prm.r) return fail(c, BGV_E_PTXT_MOD, "less_than takes values tagged t = p^r");
  return guarded(c, [&] {
    return deliver(c, ev_less_than(c, k, borrow(x), y ? borrow(y) : nullptr), out);
  });
}

BGV_EXPORT bgv_status bgv_rotate_sum(bgv_ctx* c, const bgv_keys* k, const bgv_ct* in, bgv_ct* out) {
  NEED_CTX(c);
  if (!k) return fail(c, BGV_E_NOKEY, "no keys");
  CHECK(check_in(c, in, "null input"));
  for (int i = 1; i < c->ell / 2; i *= 2)
    if (!k->galois.count(galois_elt(c, i))) return fail(c, BGV_E_NOKEY, "missing a power-of-two rotation key");
  if (!k->galois.count(galois_elt(c, BGV_ROW_SWAP))) return fail(c, BGV_E_NOKEY, "missing the row-swap key");
  return guarded(c, [&] { return deliver(c, ev_rotate_sum(c, k, borrow(in)), out); });
}

BGV_EXPORT bgv_status bgv_mul(bgv_ctx* c, const bgv_keys* k, const bgv_ct* a, const bgv_ct* b, bgv_ct* out) {
  NEED_CTX(c);
  if (!k || !k->relin) return fail(c, BGV_E_NOKEY, "no relinearisation key");
  CHECK(check_in(c, a, "null a"));
  CHECK(check_in(c, b, "null b"));
  if (a->t_exp != b->t_exp) return fail(c, BGV_E_PTXT_MOD, "operands with different plaintext moduli");
  if (a->n != b->n && a->n != 1 && b->n != 1) return fail(c, BGV_E_ARG, "batch sizes differ");
  if (std::min(a->level, b->level) < 2) return fail(c, BGV_E_LEVEL, "no level left for a product");
  return guarded(c, [&] { return deliver(c, ev_mul(c, k, borrow(a), borrow(b)), out); });
}

BGV_EXPORT bgv_status bgv_batch_sum(bgv_ctx* c, const bgv_ct* in, bgv_ct* out) {
  NEED_CTX(c);
  CHECK(check_in(c, in, "null input"));
  return guarded(c, [&] { return deliver(c, ev_batch_sum(c, borrow(in)), out); });
}

static bgv_status filter_check(bgv_ctx* c, const bgv_keys* k, const bgv_ct* a, const bgv_ct* thr, const bgv_ct* b,
                               const bgv_ct* cc) {
  if (!k || !k->relin) return fail(c, BGV_E_NOKEY, "no keys");
  CHECK(check_in(c, a, "null a"));
  CHECK(check_in(c, thr, "null thr"));
  CHECK(check_in(c, b, "null b"));
  CHECK(check_in(c, cc, "null c"));
  const int r = c->prm.r;
  if (a->t_exp != r || thr->t_exp != r || b->t_exp != r || cc->t_exp != r)
    return fail(c, BGV_E_PTXT_MOD, "the query runs on inputs tagged t = p^r");
  if (b->n != a->n || cc->n != a->n || (thr->n != 1 && thr->n != a->n)) return fail(c, BGV_E_ARG, "batch sizes differ");
  if (a->level != thr->level) return fail(c, BGV_E_LEVEL, "a and thr at different levels");
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_filter_sum(bgv_ctx* c, const bgv_keys* k, const bgv_ct* a, const bgv_ct* thr,
                                     const bgv_ct* b, const bgv_ct* cc, bgv_ct* out) {
  NEED_CTX(c);
  CHECK(filter_check(c, k, a, thr, b, cc));
  for (int i = 1; i < c->ell / 2; i *= 2)
    if (!k->galois.count(galois_elt(c, i))) return fail(c, BGV_E_NOKEY, "missing a power-of-two rotation key");
  if (!k->galois.count(galois_elt(c, BGV_ROW_SWAP))) return fail(c, BGV_E_NOKEY, "missing the row-swap key");
  return guarded(c, [&] { return deliver(c, ev_filter_sum(c, k, borrow(a), borrow(thr), borrow(b), borrow(cc)), out); });
}

BGV_EXPORT bgv_status bgv_filter_products(bgv_ctx* c, const bgv_keys* k, const bgv_ct* a, const bgv_ct* thr,
                                          const bgv_ct* b, const bgv_ct* cc, bgv_ct* out) {
  NEED_CTX(c);
  CHECK(filter_check(c, k, a, thr, b, cc));
  return guarded(c, [&] {
    return deliver(c, ev_filter_products(c, k, borrow(a), borrow(thr), borrow(b), borrow(cc)), out);
  });
}

static bgv_status filter_and_args(bgv_ctx* c, const bgv_keys* k, int32_t n_pred, const bgv_ct* cols,
                                  const bgv_ct* thrs, const int32_t* ops, const bgv_ct* b, const bgv_ct* cc,
                                  std::vector<CipherP>& vc, std::vector<CipherP>& vt, std::vector<int>& vo) {
  if (!k || !k->relin) return fail(c, BGV_E_NOKEY, "no keys");
  if (n_pred < 1 || n_pred > 16 || !cols || !thrs || !ops) return fail(c, BGV_E_ARG, "1 to 16 predicates");
  CHECK(check_in(c, b, "null b"));
  CHECK(check_in(c, cc, "null c"));
  const int r = c->prm.r;
  if (b->t_exp != r || cc->t_exp != r) return fail(c, BGV_E_PTXT_MOD, "the query runs on inputs tagged t = p^r");
  if (cc->n != b->n) return fail(c, BGV_E_ARG, "batch sizes differ");
  for (int i = 0; i < n_pred; ++i) {
    CHECK(check_in(c, &cols[i], "null column"));
    CHECK(check_in(c, &thrs[i], "null threshold"));
    if (ops[i] < BGV_OP_LT || ops[i] > BGV_OP_NEQ) return fail(c, BGV_E_ARG, "bad predicate op");
    if (cols[i].t_exp != r || thrs[i].t_exp != r) return fail(c, BGV_E_PTXT_MOD, "predicates compare values tagged t = p^r");
    if (cols[i].n != b->n || (thrs[i].n != 1 && thrs[i].n != b->n)) return fail(c, BGV_E_ARG, "batch sizes differ");
    if (cols[i].level != thrs[i].level) return fail(c, BGV_E_LEVEL, "a column and its threshold at different levels");
    vc.push_back(borrow(&cols[i]));
    vt.push_back(borrow(&thrs[i]));
    vo.push_back(ops[i]);
  }
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_filter_and_products(bgv_ctx* c, const bgv_keys* k, int32_t n_pred, const bgv_ct* cols,
                                              const bgv_ct* thrs, const int32_t* ops, const bgv_ct* b, const bgv_ct* cc,
                                              bgv_ct* out) {
  NEED_CTX(c);
  std::vector<CipherP> vc, vt;
  std::vector<int> vo;
  CHECK(filter_and_args(c, k, n_pred, cols, thrs, ops, b, cc, vc, vt, vo));
  return guarded(c, [&] { return deliver(c, ev_filter_and_products(c, k, vc, vt, vo, borrow(b), borrow(cc)), out); });
}

BGV_EXPORT bgv_status bgv_filter_and_sum(bgv_ctx* c, const bgv_keys* k, int32_t n_pred, const bgv_ct* cols,
                                         const bgv_ct* thrs, const int32_t* ops, const bgv_ct* b, const bgv_ct* cc,
                                         bgv_ct* out) {
  NEED_CTX(c);
  std::vector<CipherP> vc, vt;
  std::vector<int> vo;
  CHECK(filter_and_args(c, k, n_pred, cols, thrs, ops, b, cc, vc, vt, vo));
  for (int i = 1; i < c->ell / 2; i *= 2)
    if (!k->galois.count(galois_elt(c, i))) return fail(c, BGV_E_NOKEY, "missing a power-of-two rotation key");
  if (!k->galois.count(galois_elt(c, BGV_ROW_SWAP))) return fail(c, BGV_E_NOKEY, "missing the row-swap key");
  return guarded(c, [&] { return deliver(c, ev_filter_and_sum(c, k, vc, vt, vo, borrow(b), borrow(cc)), out); });
}

BGV_EXPORT bgv_status bgv_relu(bgv_ctx* c, const bgv_keys* k, const bgv_ct* x, bgv_ct* out) {
  NEED_CTX(c);
  if (!k || !k->relin) return fail(c, BGV_E_NOKEY, "no keys");
  CHECK(check_in(c, x, "null x"));
  if (x->t_exp != c->prm.r) return fail(c, BGV_E_PTXT_MOD, "the input must be tagged t = p^r");
  return guarded(c, [&] { return deliver(c, ev_relu(c, k, borrow(x)), out); });
}

BGV_EXPORT bgv_status bgv_ntt(bgv_ctx* c, uint64_t* d, int64_t cap_words, int32_t n_polys, int32_t level,
                              int32_t inverse) {
  NEED_CTX(c);
  if (!d || n_polys < 1 || level < 1 || level > c->Ltot) return fail(c, BGV_E_ARG, "bad ntt arguments");
  if (cap_words < (int64_t)n_polys * level * c->N) return fail(c, BGV_E_ARG, "buffer too small");
  if ((int64_t)n_polys * level > 65535) return fail(c, BGV_E_ARG, "more than 65535 limbs in one call");
  return guarded(c, [&] {
    op_ntt(c, d, n_polys, level, inverse != 0);
    return BGV_OK;
  });
}

BGV_EXPORT bgv_status bgv_set_ntt_chunk(bgv_ctx* c, int32_t limbs) {
  NEED_CTX(c);
  if (limbs < 0) return fail(c, BGV_E_ARG, "chunk must be >= 0");
  c->ntt_chunk = limbs;
  return BGV_OK;
}

BGV_EXPORT int32_t bgv_get_ntt_chunk(const bgv_ctx* c) { return c ? c->ntt_chunk : 0; }

BGV_EXPORT bgv_status bgv_trim(bgv_ctx* c, int64_t* held_bytes) {
  NEED_CTX(c);
  hipError_t e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) {
    c->err = std::string("device error: ") + hipGetErrorString(e);
    return BGV_E_DEVICE;
  }
  c->pool.trim();
  if (held_bytes) *held_bytes = (int64_t)c->pool.held;
  return BGV_OK;
}

struct bgv_graph {
  bgv_ctx* ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

BGV_EXPORT bgv_status bgv_capture_begin(bgv_ctx* c) {
  NEED_CTX(c);
  if (c->capturing) return fail(c, BGV_E_ARG, "already capturing");
  // capture on a stream of the library's own (the context stream may be the null
  // stream, which cannot be captured); the graph is launched on the context stream
  hipError_t e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
  if (e == hipSuccess && !c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    c->err = std::string("capture begin: ") + hipGetErrorString(e);
    return BGV_E_DEVICE;
  }
  c->saved_stream = c->stream;
  c->stream = c->cap_stream;
  c->capturing = true;
  c->graphs_alive += 1;  // keep scratch reserved from the start of the capture
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_capture_end(bgv_ctx* c, bgv_graph** out) {
  NEED_CTX(c);
  if (!c->capturing || !out) return fail(c, BGV_E_ARG, "not capturing");
  c->capturing = false;
  bgv_graph* g = new (std::nothrow) bgv_graph();
  if (!g) {
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(c->cap_stream, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    c->stream = c->saved_stream;
    c->graphs_alive -= 1;
    return BGV_E_OOM;
  }
  g->ctx = c;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g->graph);
  c->stream = c->saved_stream;
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    c->err = std::string("graph capture: ") + hipGetErrorString(e);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    c->graphs_alive -= 1;
    return BGV_E_DEVICE;
  }
  *out = g;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_graph_launch(bgv_ctx* c, const bgv_graph* g) {
  NEED_CTX(c);
  if (!g || g->ctx != c) return fail(c, BGV_E_ARG, "graph of another context");
  hipError_t e = hipGraphLaunch(g->exec, c->stream);
  if (e != hipSuccess) {
    c->err = std::string("hipGraphLaunch: ") + hipGetErrorString(e);
    return BGV_E_DEVICE;
  }
  return BGV_OK;
}

BGV_EXPORT void bgv_graph_destroy(bgv_graph* g) {
  if (!g) return;
  if (g->ctx && g->ctx->stream) (void)hipStreamSynchronize(g->ctx->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->ctx) g->ctx->graphs_alive -= 1;
  delete g;
}

BGV_EXPORT bgv_status bgv_set_schedule(bgv_ctx* c, int32_t schedule) {
  NEED_CTX(c);
  if (schedule != BGV_SCHED_FAST && schedule != BGV_SCHED_BASIC) return fail(c, BGV_E_ARG, "unknown schedule");
  c->schedule = schedule;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_set_ntt_split(bgv_ctx* c, int32_t s) {
  NEED_CTX(c);
  if (s != 0 && (s < 4 || s > 8 || c->logN - s < 4 || c->logN - s > 8 || c->logN <= 8))
    return fail(c, BGV_E_ARG, "split out of range");
  c->ntt_split = s;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_autotune_ntt(bgv_ctx* c, int32_t limbs, int32_t reps, int32_t* best_split, float* best_us) {
  NEED_CTX(c);
  if (limbs < 1 || reps < 1) return fail(c, BGV_E_ARG, "limbs and reps must be positive");
  if (limbs > 65535) return fail(c, BGV_E_ARG, "more than 65535 limbs in one call");
  if (c->capturing) return fail(c, BGV_E_ARG, "cannot tune while capturing");
  return guarded(c, [&] {
    std::vector<int> cands;
    if (c->logN <= 8) cands.push_back(0);
    for (int s = 4; s <= 8 && c->logN > 8; ++s)
      if (c->logN - s >= 4 && c->logN - s <= 8) cands.push_back(s);
    // zero residues are valid input; the transform's time does not depend on the values
    Scratch buf(c, (size_t)limbs * c->N);
    if (hipMemsetAsync(buf.d, 0, buf.bytes, c->stream) != hipSuccess) throw OpError{BGV_E_DEVICE};
    // events and the split setting are restored on every exit, exceptions included
    struct Ev {
      hipEvent_t e = nullptr;
      ~Ev() {
        if (e) (void)hipEventDestroy(e);
      }
    } ev0, ev1;
    if (hipEventCreate(&ev0.e) != hipSuccess || hipEventCreate(&ev1.e) != hipSuccess) throw OpError{BGV_E_DEVICE};
    hipEvent_t e0 = ev0.e, e1 = ev1.e;
    const int saved = c->ntt_split;
    struct Restore {
      int& split;
      int value;
      ~Restore() { split = value; }
    } restore{c->ntt_split, saved};
    int best = saved;
    float best_t = 1e30f;
    const int L = c->prm.L;
    for (int s : cands) {
      c->ntt_split = s;
      lk::ntt(c, buf.d, limbs, LimbMap{L, L, L, 0, 1, 0, 0}, false);  // warm-up
      (void)hipEventRecord(e0, c->stream);
      for (int r = 0; r < reps; ++r) lk::ntt(c, buf.d, limbs, LimbMap{L, L, L, 0, 1, 0, 0}, false);
      (void)hipEventRecord(e1, c->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const float us = ms * 1000.f / reps;
      if (us < best_t) {
        best_t = us;
        best = s;
      }
    }
    restore.value = best >= 0 ? best : saved;
    if (best_split) *best_split = restore.value;
    if (best_us) *best_us = best_t;
    return BGV_OK;
  });
}

BGV_EXPORT bgv_status bgv_get_stats(const bgv_ctx* c, bgv_stats* o) {
  if (!c || !o) return BGV_E_ARG;
  o->key_switches = c->stats.key_switches;
  o->rescale_drops = c->stats.rescale_drops;
  o->limb_drops = c->stats.limb_drops;
  o->odd_splits = c->stats.odd_splits;
  o->algo_bytes = c->stats.algo_bytes;
  o->max_baby_k = c->stats.max_baby_k;
  o->max_inner_terms = c->stats.max_inner_terms;
  o->max_inner_outputs = c->stats.max_inner_outputs;
  o->max_tensor_pairs = c->stats.max_tensor_pairs;
  return BGV_OK;
}

BGV_EXPORT bgv_status bgv_reset_stats(bgv_ctx* c) {
  NEED_CTX(c);
  c->stats = Stats{};
  return BGV_OK;
}
