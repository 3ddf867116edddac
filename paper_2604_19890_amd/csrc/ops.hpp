// Internal operation layer: owned temporaries, the operations behind the C-ABI,
// the polynomial evaluator and the space-switching composites.
#pragma once
#include <memory>
#include <vector>

#include "ctx.hpp"

bgv_status ctx_build(bgv_ctx* c, const bgv_params* prm, hipStream_t stream);
void ctx_free(bgv_ctx* c);
bool build_encoder(bgv_ctx* c);

// A ciphertext batch view (no ownership).
struct CtV {
  uint64_t* d = nullptr;
  int n = 0, level = 0, t_exp = 0;
  // limbs per polynomial in memory when the batch is a view of the lower `level` limbs of a
  // deeper one (0: level).  Only the tensor kernels and the inner sums read views.
  int stride = 0;
  int nz = 0;  // noise estimate, sixteenths of a bit (0: unknown)
};
inline int lstride(const CtV& v) { return v.stride ? v.stride : v.level; }

// Device scratch from the context pool, returned on destruction.
struct Scratch {
  bgv_ctx* c = nullptr;
  uint64_t* d = nullptr;
  size_t bytes = 0;
  Scratch() = default;
  Scratch(bgv_ctx* cc, size_t words);
  ~Scratch();
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
};

// An owned ciphertext batch.
struct Cipher {
  std::shared_ptr<Scratch> buf;  // shared by views that differ only in the t_exp tag
  CtV v;
};
typedef std::shared_ptr<Cipher> CipherP;

struct OpError {
  bgv_status st;
};

CipherP new_cipher(bgv_ctx* c, int n, int level, int t_exp);
CipherP clone(bgv_ctx* c, const CtV& x);
inline size_t ct_words(const bgv_ctx* c, int level) { return (size_t)2 * level * c->N; }

// ---- primitive operations (enqueue on the context stream; no argument checks)
void op_ntt(bgv_ctx* c, uint64_t* d, int n_polys, int level, bool inverse);
void op_add_sub(bgv_ctx* c, const CtV& a, const CtV& b, const CtV& out, int op);
void op_negate(bgv_ctx* c, const CtV& a, const CtV& out);
void op_mul_scalar(bgv_ctx* c, const CtV& a, int64_t k, const CtV& out);
void op_add_const(bgv_ctx* c, const CtV& a, int64_t k, const CtV& out);
void op_divide_by_p(bgv_ctx* c, const CtV& a, const CtV& out);
void op_mul_relin(bgv_ctx* c, const bgv_keys* keys, const CtV& a, const CtV& b, const CtV& out);
void op_rotate(bgv_ctx* c, const bgv_keys* keys, const CtV& in, int g, const CtV& out);
void op_mul_ms(bgv_ctx* c, const bgv_keys* keys, const CtV& a, const CtV& b, const CtV& out);  // product + one switch
void op_mod_switch(bgv_ctx* c, const CtV& in, const CtV& out);         // one prime
// the same with caller-provided scratch T [n][2][N] and W [n][2][level-1][N] (no allocation)
void op_mod_switch_with(bgv_ctx* c, const CtV& in, const CtV& out, uint64_t* T, uint64_t* W);
void op_mod_switch_to(bgv_ctx* c, const CtV& in, int to, const CtV& out);  // repeated
void op_copy(bgv_ctx* c, const CtV& in, const CtV& out);
int galois_elt(const bgv_ctx* c, int step);

bgv_status op_encrypt(bgv_ctx* c, const int8_t* s, const uint64_t* slots, const uint64_t* c1, const int32_t* e,
                      const CtV& out);
bgv_status op_decrypt(bgv_ctx* c, const int8_t* s, const CtV& in, uint64_t* slots, uint8_t* nonconst);
bgv_status op_keygen(bgv_ctx* c, const int8_t* s, const uint64_t* a, const int32_t* e, const std::vector<int>& gal,
                     bgv_keys* keys);

// ---- noise estimate (sixteenths of a bit; 0 = unknown, and unknown in gives unknown out)
void noise_init(bgv_ctx* c);
int nz_lgc(uint64_t x);  // ceil(16 log2 x)
int nz_lgf(uint64_t x);  // floor(16 log2 x)
int nz_add(int a, int b);
int nz_sum_of(int a, int n);
int nz_scalar(int a, int64_t k_centered);
int nz_add_const(int a, int64_t k_centered);
int nz_divide_by_p(const bgv_ctx* c, int a);
int nz_switch(const bgv_ctx* c, int a, int t_exp);
int nz_tensor(const bgv_ctx* c, int a, int b);
int nz_key_switch(const bgv_ctx* c, int a, int t_exp, int level);
int nz_mul_ms(const bgv_ctx* c, int a, int b, int t_exp, int level);  // product at `level`, one switch

// ---- evaluator and composites (owned results)
CipherP ev_align(bgv_ctx* c, const CipherP& x, int level);
CipherP ev_materialize(bgv_ctx* c, const CipherP& x);  // a contiguous batch (copies a view's limbs)
CipherP ev_mul(bgv_ctx* c, const bgv_keys* k, const CipherP& a, const CipherP& b);
CipherP ev_add(bgv_ctx* c, const CipherP& a, const CipherP& b);
CipherP ev_eval_poly(bgv_ctx* c, const bgv_keys* k, const CipherP& x, const std::vector<int64_t>& coeffs,
                     std::vector<CipherP>* giant_out = nullptr, int* giant_k = nullptr);
std::vector<CipherP> ev_space_reduce(bgv_ctx* c, const bgv_keys* k, const CipherP& x);
CipherP ev_compare(bgv_ctx* c, const bgv_keys* k, const std::vector<CipherP>& digits, int op);
CipherP ev_space_raise(bgv_ctx* c, const bgv_keys* k, const CipherP& x);
CipherP ev_rotate_sum(bgv_ctx* c, const bgv_keys* k, const CipherP& x);
CipherP ev_less_than(bgv_ctx* c, const bgv_keys* k, const CipherP& x, const CipherP& y);
CipherP ev_batch_sum(bgv_ctx* c, const CipherP& x);
CipherP ev_filter_products(bgv_ctx* c, const bgv_keys* k, const CipherP& a, const CipherP& thr, const CipherP& b,
                           const CipherP& cc);
CipherP ev_filter_sum(bgv_ctx* c, const bgv_keys* k, const CipherP& a, const CipherP& thr, const CipherP& b,
                      const CipherP& cc);
CipherP ev_relu(bgv_ctx* c, const bgv_keys* k, const CipherP& x);
CipherP ev_filter_and_products(bgv_ctx* c, const bgv_keys* k, const std::vector<CipherP>& cols,
                               const std::vector<CipherP>& thrs, const std::vector<int>& ops, const CipherP& b,
                               const CipherP& cc);
CipherP ev_filter_and_sum(bgv_ctx* c, const bgv_keys* k, const std::vector<CipherP>& cols,
                          const std::vector<CipherP>& thrs, const std::vector<int>& ops, const CipherP& b,
                          const CipherP& cc);
int eval_depth(int degree);
