/*
 * bgv.h -- C-ABI of the MI355X (gfx950) space-switching BGV library.
 *
 * The library evaluates the exact RNS arithmetic that carries every homomorphic
 * multiplication of the space-switching method (arXiv 2604.19890): negacyclic
 * NTT/INTT over 50-bit primes, pointwise modular products, hybrid key switching
 * (relinearisation and slot rotation), modulus switching, and on top of them the
 * reduction Z_{p^r} -> Z_p (Algorithm 3), the digit-wise comparison (Algorithm 4)
 * and modulus raising Z_p -> Z_{p^r} (Method, modulus-raising subsection).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Ring: Z_Q[X]/(X^N + 1), N = 2^log_n; the paper's general cyclotomic Phi_m
 *   (Background, BGV subsection) taken at m = 2N.  Plaintext modulus p^r with
 *   p = 1 (mod 4); ell = 2^(v2(p-1)-1) slots, each holding a constant of Z_{p^r}.
 * Primes: the first L + K primes below 2^50 that are 1 mod lcm(2N, p^r), in
 *   descending order; q_0..q_{L-1} carry the ciphertext, the last K are the
 *   special primes of hybrid key switching (digit size alpha = K).
 * Ciphertext batches (bgv_ct): `d` is a DEVICE buffer owned by the caller that
 *   holds `n` ciphertexts back to back, each laid out [2][level][N] as uint64
 *   residues in [0, q_i), in evaluation form (negacyclic NTT under the smallest
 *   primitive 2N-th root psi_i of q_i, bit-reversed order: word j of limb i is
 *   c(psi_i^(2 brv(j) + 1)) mod q_i).  `cap_words` is the number of uint64 words
 *   the buffer can hold; every entry point that writes a batch checks it and
 *   returns BGV_E_ARG rather than writing past it.  `t_exp` is the current
 *   plaintext-modulus exponent (t = p^t_exp).
 * Streams: every device operation is enqueued on the context's stream (a
 *   hipStream_t given at creation or by bgv_set_stream) and returns before the
 *   work completes.  Argument, level and plaintext-modulus errors are detected on
 *   the host before anything is enqueued.  Device faults surface at bgv_sync.
 *   An output batch may alias an input batch of the same operation.
 *   A context is not thread-safe; use one context per host thread.
 * Randomness: the library never samples.  Secret keys, key-switching and
 *   encryption randomness come in as host arrays from the caller's seeded
 *   generator.
 * Errors: every entry point returns a bgv_status; bgv_last_error gives a
 *   message for the last failure on a context.
 */
#ifndef BGV_H
#define BGV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BGV_OK = 0,
  BGV_E_ARG = 1,         /* null pointer, bad size, buffer too small, bad op code */
  BGV_E_PARAM = 2,       /* unsupported ring / plaintext / chain parameters     */
  BGV_E_LEVEL = 3,       /* level mismatch, or no level left to switch down      */
  BGV_E_PTXT_MOD = 4,    /* plaintext-modulus exponents differ or are invalid    */
  BGV_E_NOKEY = 5,       /* no Galois key for the requested rotation             */
  BGV_E_OOM = 6,         /* device or host allocation failed                     */
  BGV_E_DEVICE = 7,      /* a HIP runtime call failed                            */
  BGV_E_UNSUPPORTED = 8  /* no G_{p,e} table for the ciphertext's exponent e     */
} bgv_status;

typedef struct {
  int32_t log_n; /* N = 2^log_n, 4 <= log_n <= 16                                 */
  int32_t p;     /* plaintext prime, p = 1 mod 4                                  */
  int32_t r;     /* plaintext exponent, t = p^r: 1 <= r <= 4, p^r < 2^31          */
  int32_t L;     /* ciphertext primes                                             */
  int32_t K;     /* special primes for hybrid key switching; digit size alpha = K */
} bgv_params;

typedef struct {
  uint64_t* d;       /* device buffer, n x [2][level][N] uint64, evaluation form */
  int64_t cap_words; /* capacity of d in uint64 words                            */
  int32_t n;         /* ciphertexts in the batch, 1 .. bgv_info.max_batch         */
  int32_t level;     /* active primes q_0..q_{level-1}                           */
  int32_t t_exp;     /* plaintext modulus p^t_exp                                */
  int32_t noise;     /* noise estimate: log2 of a bound on the largest coefficient of
                        [c0 + c1 s]_Q (the plaintext included), in sixteenths of a bit;
                        0 = unknown.  Written by every call that writes a batch (fresh
                        encryptions get lgc(20 t)); read by the evaluator to decide how
                        an operand reaches a lower level (below).  A batch assembled by
                        the caller should carry the largest estimate of its parts, or 0 */
} bgv_ct;

typedef struct {
  int32_t N, log_n, p, r, L, K, alpha, dnum; /* dnum = ceil(L / alpha)       */
  int32_t slots, d;                          /* ell slots of degree d = N/ell */
  int64_t t;                                 /* p^r                          */
  int32_t max_batch; /* largest n one call accepts: every launch of the call fits the
                        grid limits (n * max(dnum, 2) * (L + K) <= 65535); larger
                        batches are split by the caller, a call above it fails with
                        BGV_E_ARG                                                      */
  int32_t _pad;
} bgv_info;

typedef struct bgv_ctx bgv_ctx;
typedef struct bgv_keys bgv_keys;

#define BGV_ROW_SWAP (-1) /* rotation step that swaps the two slot rows (X -> X^(2N-1)) */
#define BGV_OP_LT 0  /* [value < 0] on the centered range of Z_{p^r}          */
#define BGV_OP_EQ 1  /* [value = 0]                                          */
#define BGV_OP_GT 2  /* [value > 0]: digit polynomial F_GT(x) = F_LT(-x)      */
#define BGV_OP_LE 3  /* 1 - GT                                               */
#define BGV_OP_GE 4  /* 1 - LT                                               */
#define BGV_OP_NEQ 5 /* 1 - EQ                                               */

/* ---- context -------------------------------------------------------------
 * bgv_ctx_create: derives the prime chain, NTT roots and twiddles, slot roots,
 *   base-conversion constants and the coefficient tables of G_{p,2}, F_LT, F_EQ,
 *   and uploads the device tables.  `hip_stream` is a hipStream_t (NULL = the
 *   null stream).  BGV_E_PARAM for unsupported parameters (p = 3 mod 4, ring too
 *   small for p, not enough 50-bit primes, L + K > 64).  The context owns all of
 *   its memory; bgv_ctx_destroy frees it (after synchronising its stream).     */
bgv_status bgv_ctx_create(const bgv_params* prm, void* hip_stream, bgv_ctx** out);
void bgv_ctx_destroy(bgv_ctx* ctx);
bgv_status bgv_set_stream(bgv_ctx* ctx, void* hip_stream);
bgv_status bgv_ctx_info(const bgv_ctx* ctx, bgv_info* out);
/* primes (L + K values, q_0..q_{L-1} then the special primes) into host `out` */
bgv_status bgv_ctx_primes(const bgv_ctx* ctx, uint64_t* out);
/* words of one ciphertext at `level` (2 * level * N) */
int64_t bgv_ct_words(const bgv_ctx* ctx, int32_t level);
bgv_status bgv_sync(bgv_ctx* ctx);
const char* bgv_last_error(const bgv_ctx* ctx);
/* bgv_trim: synchronise the stream and free the context's cached scratch buffers
 * (device memory the library keeps for reuse between operations); `held_bytes`, if not
 * NULL, receives the bytes still held (buffers in use) afterwards.                  */
bgv_status bgv_trim(bgv_ctx* ctx, int64_t* held_bytes);

/* ---- keys ----------------------------------------------------------------
 * Hybrid key-switching keys (digit j = primes j*alpha .. min((j+1)*alpha, L)-1):
 *   ksk_j = (b_j, a_j),  b_j = -a_j s + t e_j + [prime in digit j] P s'  (mod every
 *   one of the L + K primes, P = product of the special primes), with s' = s^2 for
 *   relinearisation and s' = s(X^g) for the Galois element g of a rotation.
 * Host inputs: s [N] ternary; a [n_keys][dnum][L+K][N] residues (< the prime of
 *   their row); e [n_keys][dnum][N] small signed errors.  Key order: relinearisation,
 *   then one key per entry of `steps` (row rotation by steps[i] slots, i.e.
 *   g = 5^steps[i] mod 2N; BGV_ROW_SWAP allowed), then the row swap if with_conj.
 * Keys live in device memory owned by the returned object (evaluation form).  */
bgv_status bgv_keygen(bgv_ctx* ctx, const int8_t* s, const uint64_t* a, const int32_t* e,
                      const int32_t* steps, int32_t n_steps, int32_t with_conj, bgv_keys** out);
void bgv_keys_destroy(bgv_keys* keys);
int64_t bgv_keys_bytes(const bgv_keys* keys);

/* ---- encryption (Algorithm 1) and decryption (Algorithm 2) ---------------
 * bgv_encrypt: out->n ciphertexts at level L with t = p^r.  Host inputs per
 *   ciphertext b: slots[b*ell ..] values mod p^r (encoded as m(X) = M(X^d), M the
 *   interpolant of the slots at the slot roots, coefficients lifted to the
 *   centered range); c1[b] [L][N] uniform residues; e[b] [N] small errors.
 *   c0 = m + t e - c1 s.  s is host [N] ternary.
 * bgv_decrypt: synchronises the stream, then writes in->n * ell slot values
 *   (mod p^t_exp) to host `slots`; if `nonconst` is not NULL it receives one flag
 *   per slot that is 1 when the slot is not a constant of Z_{p^t_exp}.          */
bgv_status bgv_encrypt(bgv_ctx* ctx, const int8_t* s, const uint64_t* slots, const uint64_t* c1,
                       const int32_t* e, bgv_ct* out);
bgv_status bgv_decrypt(bgv_ctx* ctx, const int8_t* s, const bgv_ct* in, uint64_t* slots,
                       uint8_t* nonconst);

/* ---- linear operations (slot-wise) ----------------------------------------
 * add/sub need equal level (BGV_E_LEVEL) and t_exp (BGV_E_PTXT_MOD); b may be a
 * single ciphertext (b->n == 1) broadcast against a batch.  Constants are lifted
 * to the centered range mod p^t_exp.  bgv_add_const adds c to every slot.
 * bgv_divide_by_p: DivideByP (Method, reduction subsection) -- multiply by
 * p^-1 mod each q_i and lower t_exp by one; the caller guarantees every slot is
 * 0 mod p.  bgv_set_t_exp changes only the tag: ChangeModToP (t_exp = 1, Lemma 4)
 * or the first half of modulus raising (t_exp = r).                           */
bgv_status bgv_add(bgv_ctx* ctx, const bgv_ct* a, const bgv_ct* b, bgv_ct* out);
bgv_status bgv_sub(bgv_ctx* ctx, const bgv_ct* a, const bgv_ct* b, bgv_ct* out);
bgv_status bgv_negate(bgv_ctx* ctx, const bgv_ct* a, bgv_ct* out);
bgv_status bgv_mul_scalar(bgv_ctx* ctx, const bgv_ct* a, int64_t c, bgv_ct* out);
bgv_status bgv_add_const(bgv_ctx* ctx, const bgv_ct* a, int64_t c, bgv_ct* out);
bgv_status bgv_divide_by_p(bgv_ctx* ctx, const bgv_ct* a, bgv_ct* out);
bgv_status bgv_set_t_exp(bgv_ctx* ctx, bgv_ct* ct, int32_t t_exp);

/* ---- products, rotations, modulus switching -------------------------------
 * bgv_mul_relin: tensor product and relinearisation by hybrid key switching
 *   (ModUp of each digit, inner product with the key, ModDown with the t-corrected
 *   delta); output at the input level, no modulus switch inside.
 * bgv_rotate: X -> X^g on both components, then key switching of the second under
 *   the Galois key (BGV_E_NOKEY if no key for the step).
 * bgv_mod_switch: drop the top prime: w = centered([c_top t^-1]_{q_top}),
 *   c_i <- (c_i - t w) q_top^-1.  BGV_E_LEVEL at level 1.
 * bgv_mod_switch_to: the same single-prime step repeated down to `level`
 *   (bit-identical to repeated bgv_mod_switch, computed in one fused pass).     */
bgv_status bgv_mul_relin(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* a, const bgv_ct* b,
                         bgv_ct* out);
bgv_status bgv_rotate(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* in, int32_t step,
                      bgv_ct* out);
bgv_status bgv_mod_switch(bgv_ctx* ctx, const bgv_ct* in, bgv_ct* out);
bgv_status bgv_mod_switch_to(bgv_ctx* ctx, const bgv_ct* in, int32_t level, bgv_ct* out);

/* ---- polynomial evaluation and space switching ----------------------------
 * bgv_eval_poly: sum_i coeffs[i] x^i (coefficients reduced mod p^t_exp) by the
 *   baby-step/giant-step Paterson-Stockmeyer form (Theorem 2), in the context's
 *   schedule (bgv_set_schedule); every relinearisation is followed by one modulus
 *   switch.  The output level is input level minus the schedule depth (the same in
 *   both schedules); BGV_E_LEVEL if the chain is too short.
 * bgv_set_schedule: the evaluation schedule of every polynomial of the context, the
 *   space-switching operations included (the paper fixes only the Paterson-Stockmeyer
 *   form).  Both form baby powers x^2..x^k and giant powers y^j, y = x^k, with
 *   x^i = (x^(i/2))^2 for i a power of two, else x^h x^(i-h) (h the largest power of two
 *   below i); each product first brings its operands to the lower level, as does
 *   each addition.
 *   BGV_SCHED_FAST (0, the default): odd-structured polynomials (every even
 *   coefficient strictly between the constant and the leading term zero) take k =
 *   the smallest power of two with k^2 >= D + 1, others 2k^2 >= D + 1; only the baby
 *   powers the inner sums need (closed under the power rule) are formed, the powers of
 *   two and the giants first, then each other one at the level its consumers need
 *   (the giants' lowest level F among the non-constant inner sums for the inner sums,
 *   one level above each power it is the second operand of); inner sums
 *   are formed at the level where the outer products meet (or lower); the products
 *   I_j y^j are aligned to their lowest common level, their tensor products summed
 *   and relinearised once, then switched once; then c_jk y^j for constant I_j in
 *   increasing j, then I_0.  An operand reaches a lower level by its noise estimate
 *   (bgv_ct.noise): while the estimate is more than 4 bits above the floor a modulus
 *   switch leaves (lgc(3 t) - 16 + 8 log2 N), one switch of the top prime; the limbs
 *   left above the target level are dropped without rescaling (the decryption
 *   relation holds modulo every divisor of the modulus and the primes are 1 mod t).
 *   An operand without an estimate (noise 0) is switched all the way.
 *   BGV_SCHED_BASIC (1): k = the smallest power of two with 2k^2 >= D + 1 for every
 *   polynomial; inner sums at the lowest level among their powers; in increasing j,
 *   I_j y^j as one product (align, relinearise, switch) or c_jk y^j, added to the
 *   running sum at the lower level; then I_0.  Every operand reaches a lower level by
 *   single-prime switches.  BGV_E_ARG for other values.
 * bgv_space_reduce: Algorithm 3 on a value tagged t = p^e (1 <= e <= r): e - 1 rounds
 *   of digits[i] = G_{p,e-i}(b), b <- DivideByP(b - digits[i]) (b starts as `in`),
 *   and digits[e-1] = b, all tagged t = p (ChangeModToP); the digits are the
 *   balanced base-p digits of each slot, least significant first.  `digits` has e
 *   entries.  G_{p,e} (Lemma 3) for e >= 3 is lifted from G_{p,e-1} one digit at
 *   a time, which needs e <= p; a context whose r exceeds p fails at creation.
 * bgv_compare: Algorithm 4 on r digit batches (least significant first), op one of
 *   BGV_OP_LT / GT (digit polynomial and the aggregation LT = LT + EQ * LT_i),
 *   BGV_OP_EQ (product of the digit equalities) or the complements LE = 1 - GT,
 *   GE = 1 - LT, NEQ = 1 - EQ (the comparison subsection's predicate family).
 * bgv_space_raise: RaiseModToP2R -- tag t = p^r, then G_{p,r}; a slot holding k
 *   mod p becomes centered_p(k) mod p^r.
 * bgv_less_than: reduce -> compare(LT) -> raise of (x - y), or of x if y is NULL;
 *   x (and y) tagged t = p^r (BGV_E_PTXT_MOD otherwise).
 * bgv_rotate_sum: every slot receives the sum of all slots (row rotations by
 *   1, 2, 4, .., ell/4 and the row swap; all those keys are needed).           */
bgv_status bgv_eval_poly(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* in, const int64_t* coeffs,
                         int32_t degree, bgv_ct* out);
#define BGV_SCHED_FAST 0
#define BGV_SCHED_BASIC 1
bgv_status bgv_set_schedule(bgv_ctx* ctx, int32_t schedule);
bgv_status bgv_space_reduce(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* in, bgv_ct* digits);
bgv_status bgv_compare(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* digits, int32_t r, int32_t op,
                       bgv_ct* out);
bgv_status bgv_space_raise(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* in, bgv_ct* out);
bgv_status bgv_less_than(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* x, const bgv_ct* y,
                         bgv_ct* out);
bgv_status bgv_rotate_sum(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* in, bgv_ct* out);

/* ---- workload glue ---------------------------------------------------------
 * bgv_mul: the evaluator's product step: both operands are brought to the lower
 *   level (as in the context's schedule, bgv_set_schedule), multiplied and
 *   relinearised, then switched down one prime (output level = min level - 1).  b may
 *   be a single ciphertext broadcast against a batch.
 * bgv_batch_sum: out (one ciphertext) = sum of the in->n ciphertexts of a batch;
 *   its noise estimate is the batch's plus ceil(16 log2 n) (n terms, each bounded by
 *   the batch's estimate).
 * bgv_filter_sum: the filter-and-aggregate query SUM(b*c WHERE a < thr) over the
 *   rows packed in the slots of the batches a, b, c (thr: one ciphertext, or a batch
 *   of the same size): per ciphertext [a < thr] * (b * c) with the product steps
 *   above, the batch summed, then rotate-and-sum so that every slot of `out` holds
 *   the total (Figure 1's WHERE -> multiply -> SUM pipeline).  In the fast schedule
 *   b * c is formed one level above the predicate's result, from b and c brought down
 *   first (in the basic one, at their own level).  Needs the keys of bgv_rotate_sum.
 * bgv_relu: x * (1 - [x < 0]) slot-wise (the ReLU-style sign/compare workload).   */
bgv_status bgv_mul(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* a, const bgv_ct* b, bgv_ct* out);
bgv_status bgv_batch_sum(bgv_ctx* ctx, const bgv_ct* in, bgv_ct* out);
bgv_status bgv_filter_sum(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* a, const bgv_ct* thr, const bgv_ct* b,
                          const bgv_ct* c, bgv_ct* out);
bgv_status bgv_relu(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* x, bgv_ct* out);
/* bgv_filter_products: the per-ciphertext part of bgv_filter_sum, [a < thr] * (b * c) for
 *   each ciphertext of the batch (no sum, no rotation); thr is one ciphertext or a batch of
 *   the same size.  A serving loop sums the products of each query itself, so ciphertexts of
 *   several queries can share one batch.                                                   */
bgv_status bgv_filter_products(bgv_ctx* ctx, const bgv_keys* keys, const bgv_ct* a, const bgv_ct* thr,
                               const bgv_ct* b, const bgv_ct* c, bgv_ct* out);

/* bgv_filter_and_products / bgv_filter_and_sum: the multi-predicate query
 *   SUM(b*c WHERE col_0 op_0 thr_0 AND col_1 op_1 thr_1 AND ..) (the comparison subsection's
 *   predicate family combined by conjunction, as range filters need: lo <= a AND a < hi).
 *   Predicate i compares cols[i] with thrs[i] (one ciphertext, or a batch of the same size):
 *   ops[i] is BGV_OP_LT / LE / GT / GE / EQ / NEQ applied to cols[i] - thrs[i] (so BGV_OP_LT
 *   is [col < thr]).  Each predicate is reduced and compared in the digit space; the 0/1
 *   results are multiplied there in a balanced tree over the predicates in their order
 *   (pairs (0,1), (2,3), .., then pairs of those), raised once and multiplied by b * c
 *   (in the fast schedule formed one level above the raised result, as in bgv_filter_sum).
 *   The depth is one reduce, compare and raise plus ceil(log2 n_pred) products, so the chain
 *   must be that much longer than the single-predicate query's (BGV_E_LEVEL otherwise).
 *   1 <= n_pred <= 16.  _products gives the per-ciphertext result, _sum the batch summed and
 *   rotated so that every slot holds the total (needs the keys of bgv_rotate_sum).          */
bgv_status bgv_filter_and_products(bgv_ctx* ctx, const bgv_keys* keys, int32_t n_pred, const bgv_ct* cols,
                                   const bgv_ct* thrs, const int32_t* ops, const bgv_ct* b, const bgv_ct* c,
                                   bgv_ct* out);
bgv_status bgv_filter_and_sum(bgv_ctx* ctx, const bgv_keys* keys, int32_t n_pred, const bgv_ct* cols,
                              const bgv_ct* thrs, const int32_t* ops, const bgv_ct* b, const bgv_ct* c, bgv_ct* out);

/* ---- graph capture ---------------------------------------------------------
 * bgv_capture_begin / bgv_capture_end record every device operation the context
 * enqueues in between into an executable graph (capture in relaxed mode on a
 * stream of the library's own, after the context stream has drained; work that
 * is not the library's is not recorded); bgv_graph_launch replays it on the context's
 * stream with the same buffers (inputs, outputs, and the library's scratch, which
 * stays reserved while any graph of the context exists).  Only asynchronous
 * operations can be captured (not keygen, encrypt, decrypt, trim); run the sequence
 * once before capturing it so that its tables are built.  BGV_E_DEVICE if the
 * runtime rejects the capture.                                                   */
typedef struct bgv_graph bgv_graph;
bgv_status bgv_capture_begin(bgv_ctx* ctx);
bgv_status bgv_capture_end(bgv_ctx* ctx, bgv_graph** out);
bgv_status bgv_graph_launch(bgv_ctx* ctx, const bgv_graph* graph);
void bgv_graph_destroy(bgv_graph* graph);

/* ---- tuning ---------------------------------------------------------------
 * bgv_set_ntt_chunk: two-pass NTTs over many limbs run in chunks of `limbs`
 *   limbs (first and second pass per chunk) so that the first pass's output is
 *   still cached when the second pass reads it; 0 runs all limbs in one launch
 *   pair.  Results are identical for every setting.  BGV_E_ARG if limbs < 0.
 * bgv_get_ntt_chunk: the current setting.                                       */
bgv_status bgv_set_ntt_chunk(bgv_ctx* ctx, int32_t limbs);
int32_t bgv_get_ntt_chunk(const bgv_ctx* ctx);
/* bgv_set_modup_fused: key switching with ModUp fused into the transform passes around
 *   it (1, the default, for rings with two-pass transforms whose first pass has 5..8
 *   stages and digits of 1, 2, 4 or 6 primes: x's last inverse pass, ModUp and the first
 *   forward pass of every ModUp row run in one kernel, so neither x's coefficient form nor
 *   the untransformed ModUp rows are stored) or ModUp between full transforms (0).
 *   Results are identical either way.                                                 */
bgv_status bgv_set_modup_fused(bgv_ctx* ctx, int32_t on);
/* bgv_set_moddown_fused: how the product step (bgv_mul and the evaluator's products) runs
 *   ModDown and the modulus switch after key switching, on rings with two-pass transforms
 *   whose first pass has 5..8 stages and K <= 6.  Fused, the last inverse pass of u's special
 *   and top rows, the merged correction and the first forward pass of every corrected row
 *   run in one kernel, so the correction is never stored in coefficient form.  on = 0: never
 *   fused (separate launches); 1 (the default): fused when the batch gives that kernel at
 *   least 512 blocks (16 ciphertexts at N = 2^16), below which the separate launches are
 *   faster; 2: always fused.  Other values: BGV_E_ARG.  Results are identical either way.  */
bgv_status bgv_set_moddown_fused(bgv_ctx* ctx, int32_t on);
/* bgv_set_ntt_coop: how two-pass transforms run.  mode 0 (the only one built): two
 *   launches per transform.  mode 1, a persistent launch that would keep each limb's
 *   intermediate in one XCD's L2, is switched off and returns BGV_E_UNSUPPORTED.     */
bgv_status bgv_set_ntt_coop(bgv_ctx* ctx, int32_t mode, int32_t lookahead);
/* bgv_set_ntt_split: stages in the first of the two NTT passes (each pass does 4..8
 *   stages; 0 restores the default ceil(log N / 2)).  BGV_E_ARG if out of range.
 * bgv_autotune_ntt: times every valid split on a scratch array of `limbs` limbs
 *   (`reps` forward transforms each, HIP events on the context stream), keeps the
 *   fastest in the context and reports it with its time per transform.  Results
 *   are identical for every split.  BGV_E_ARG for limbs above 65535.               */
bgv_status bgv_set_ntt_split(bgv_ctx* ctx, int32_t first_pass_stages);
bgv_status bgv_autotune_ntt(bgv_ctx* ctx, int32_t limbs, int32_t reps, int32_t* best_split, float* best_us);

/* ---- allocation-free variant ------------------------------------------------
 * For callers that cannot allocate device memory during a call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).
 * bgv_mod_switch_noalloc: the same result as bgv_mod_switch (bit for bit), but every
 *   temporary lives in a scratch array of BGV_NOALLOC_SCRATCH_WORDS uint64 words (32 MiB)
 *   that the library holds on each GPU it runs on until the process ends; the call performs
 *   no device allocation or free.  The caller passes the input and the output (out may
 *   alias in).  The switch of n ciphertexts at level l needs 2 n l N words of scratch; a
 *   larger call returns BGV_E_ARG before anything is enqueued.  All calls on one GPU share
 *   the array (contexts and streams included): calls whose execution overlaps on one GPU
 *   race on it, so callers serialise them (one stream, or events between streams).
 *   BGV_E_DEVICE if the array's address could not be resolved on this device.          */
#define BGV_NOALLOC_SCRATCH_WORDS (4 * 1024 * 1024)
bgv_status bgv_mod_switch_noalloc(bgv_ctx* ctx, const bgv_ct* in, bgv_ct* out);

/* ---- launch statistics -----------------------------------------------------
 * Host-side counters of the work a context has enqueued since its creation or the
 * last bgv_reset_stats (they are updated when work is enqueued and never wait for
 * the device).  A batch call counts once.  Tests use them to confirm which launch
 * shapes a computation reached; they have no effect on results.                 */
typedef struct {
  int64_t key_switches;      /* relinearisations and rotations                             */
  int64_t rescale_drops;     /* single-prime modulus switches (a switch by k primes adds k) */
  int64_t limb_drops;        /* alignments that remove top limbs without rescaling         */
  int64_t odd_splits;        /* polynomial evaluations that took the odd baby-step split    */
  int64_t algo_bytes;        /* algorithmic HBM bytes of the enqueued steps: each step's one
                                read of its inputs and write of its outputs (a relinearised
                                product 6 l N 8, 6 l N 8 - 2 N 8 with its switch merged in; a
                                rotation 4 l N 8; a single modulus switch (4 l - 2) N 8; linear
                                steps their inputs and outputs), per ciphertext of a batch, plus
                                the key of a key switch once per call                         */
  int32_t max_baby_k;        /* largest baby-step count k of an evaluated polynomial        */
  int32_t max_inner_terms;   /* most baby powers read by one multi-output inner-sum launch  */
  int32_t max_inner_outputs; /* most inner sums written by one such launch                  */
  int32_t max_tensor_pairs;  /* most ciphertext pairs summed by one tensor-sum launch       */
} bgv_stats;
bgv_status bgv_get_stats(const bgv_ctx* ctx, bgv_stats* out);
bgv_status bgv_reset_stats(bgv_ctx* ctx);

/* ---- raw NTT access (the transform on its own, for tests and bandwidth runs)
 * bgv_ntt: in place on a DEVICE array holding n_polys polynomials of `level` limbs
 *   each ([n_polys][level][N] uint64 residues, limb i under q_i); forward (coefficient
 *   -> evaluation form, layout as for ciphertexts) when inverse == 0, else inverse.
 *   cap_words is the capacity of d.  At most 65535 limbs (n_polys * level) per call
 *   (the grid's y extent); BGV_E_ARG beyond.                                     */
bgv_status bgv_ntt(bgv_ctx* ctx, uint64_t* d, int64_t cap_words, int32_t n_polys, int32_t level,
                   int32_t inverse);

#ifdef __cplusplus
}
#endif
#endif /* BGV_H */
