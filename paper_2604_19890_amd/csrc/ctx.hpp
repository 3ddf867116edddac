// Internal state of a context and of a key set; launcher declarations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/bgv.h"
#include "common.hpp"

// Caching device allocator.  A context runs on one stream, so a buffer returned
// to the cache may be handed out again at once: later work on the same stream
// runs after every earlier use of it.
struct DevPool {
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> all_;
  size_t held = 0;
  const int* pinned = nullptr;  // while *pinned > 0 no cached block is freed
  void* get(size_t bytes);
  void put(void* p, size_t bytes);
  void trim();
  void release();
};

// Host-side counters of what a context has enqueued (bgv_get_stats).
struct Stats {
  int64_t key_switches = 0;   // relinearisations and rotations, one per batch call
  int64_t rescale_drops = 0;  // single-prime modulus switches (k primes at once count k)
  int64_t limb_drops = 0;     // alignments by removing top limbs without rescaling
  int64_t odd_splits = 0;     // polynomial evaluations in the odd baby-step split
  int64_t algo_bytes = 0;     // algorithmic HBM bytes of the enqueued steps (see ops.cpp)
  int32_t max_baby_k = 0;
  int32_t max_inner_terms = 0;
  int32_t max_inner_outputs = 0;
  int32_t max_tensor_pairs = 0;
};

// Noise estimate model (sixteenths of a bit): the estimate of a fresh encryption, floor(16
// log2) of the smallest ciphertext prime and of p, and per plaintext exponent e the floor a
// modulus switch leaves and, per level, what one key switch adds.
constexpr int NZ_UNIT = 16;
constexpr int NZ_SLACK = 4 * NZ_UNIT;  // lowered by dropping limbs within this of the switch floor
struct NoiseModel {
  int fresh = 0, q16 = 0, lgp = 0;
  std::vector<int> floor;            // [r+1]
  std::vector<std::vector<int>> ks;  // [r+1][L+1]
};

struct bgv_ctx {
  bgv_params prm;
  int N = 0, logN = 0, ell = 0, dslot = 0, alpha = 0, dnum = 0, Ltot = 0;
  int64_t t_full = 0;
  std::vector<uint64_t> primes;  // q_0..q_{L-1}, then the K special primes
  std::vector<uint64_t> psi;     // NTT root per prime
  std::vector<int64_t> tpow;     // p^e for e = 0..r
  hipStream_t stream = nullptr;
  std::string err;
  int ntt_chunk = 0;  // limbs per chunk of a two-pass NTT (0: one launch pair for all limbs)
  int ntt_split = 0;  // stages in the first of two NTT passes (0: ceil(log N / 2))
  int schedule = 0;   // polynomial evaluation schedule (BGV_SCHED_FAST / BGV_SCHED_BASIC)
  int modup_fused = 1;  // key switching with the fused ModUp pass (1) or ModUp between full transforms (0)
  int moddown_fused = 1;  // the product step's ModDown and switch fused with the passes around them: 0 never,
                          // 1 when the batch gives the fused kernel two blocks per CU, 2 always
  int graphs_alive = 0;  // executable graphs referring to pool buffers (trim keeps them then)
  bool capturing = false;
  hipStream_t cap_stream = nullptr;    // capture happens here (default priority, non-blocking)
  hipStream_t saved_stream = nullptr;  // the context stream while capturing
  DevPool pool;
  Stats stats;
  NoiseModel nzm;
  // device address of the allocation-free variant's scratch on this context's device
  // (looked up once per device at context creation; null if the lookup failed)
  uint64_t* noalloc_scratch = nullptr;
  int device = -1;

  // device tables
  PrimeD* d_prime = nullptr;  // [Ltot]
  double* d_tw = nullptr;     // [Ltot][N]  psi^brv(k)
  double* d_itw = nullptr;    // [Ltot][N]  psi^-brv(k)
  // ModUp: for level l in [1, L] and digit j: inverse table [alpha] and
  // basis table [alpha][Ltot] (Qhat_i mod prime m), at offset modup_off(l, j)
  double* d_modup = nullptr;
  // ModUp operand scales N^-1 Qhat_i^-1 mod q_i per (level, digit, source) [L+1][dnum][alpha]
  double* d_modup_scale = nullptr;
  // ModDown: phat_inv [K], phat_mod [K][L], pinv_q [L]
  double* d_moddown = nullptr;
  // modulus switching: qinv_tab [L][L] (q_top^-1 mod q_i at [top][i])
  double* d_msw = nullptr;
  // repeated switch from `level` down to `to`: prod_{j=to}^{level-1} q_j^-1 mod q_i
  // at [(level * (L+1) + to) * L + i]
  double* d_mswpi = nullptr;
  // t-dependent scalars: tinv_tab [r+1][Ltot] (t^-1 mod prime), tmod_tab [r+1][Ltot]
  double* d_tconst = nullptr;
  // ModDown constants with the factor t P^-1 of the merged switch folded in:
  // [e][k][i] = Phat_k * p^e * P^-1 mod q_i (e <= r, k < K, i < L)
  double* d_mdfold = nullptr;

  // host copies of scalar tables used to build kernel arguments
  std::vector<double> h_tinv, h_tmod;  // [r+1][Ltot]

  // polynomial tables (ascending coefficients)
  std::vector<int64_t> g2;    // G_{p,2} mod p^2
  std::vector<std::vector<int64_t>> gpe;  // gpe[e] = G_{p,e} mod p^e for 1 <= e <= r
  std::vector<int64_t> flt;   // F_LT mod p
  std::vector<int64_t> fgt;   // F_GT mod p
  // slot structure
  std::vector<int64_t> slot_exp;  // exponent e_j of slot j (root zeta^e_j)
  int64_t zeta = 0;
  std::vector<int64_t> encoder;   // [ell][ell] inverse Vandermonde of the slot roots mod p^r
  // device tables of polynomial coefficients reduced mod every q_i ([D+1][L] doubles),
  // keyed by (t_exp, coefficients)
  std::map<std::pair<int, std::vector<int64_t>>, double*> coeff_tabs;

  size_t modup_inv_off(int level, int j) const {
    return ((size_t)(level * dnum + j)) * (size_t)alpha * (1 + Ltot);
  }
  size_t modup_basis_off(int level, int j) const { return modup_inv_off(level, j) + alpha; }
  // largest batch per call: a grid's y extent is at most 65535, and the widest launches
  // have n * dnum' * (level + K) <= n * dnum * Ltot block rows (the first NTT pass of the
  // ModUp output) or at most n * 2 * Ltot (two polynomials' rows, e.g. the top and special
  // rows of u with one digit)
  int max_batch() const { return 65535 / ((dnum > 2 ? dnum : 2) * Ltot); }
};

struct bgv_keys {
  bgv_ctx* ctx = nullptr;
  // each key: [dnum][2][Ltot][N] uint64 in evaluation form; component 0 = b, 1 = a
  uint64_t* relin = nullptr;
  std::map<int, uint64_t*> galois;  // Galois element g -> key
  int64_t bytes = 0;
};

// ------------------------------------------------------------------ launchers
namespace lk {
// stages of the first and second NTT pass (second = 0 for a single pass)
void ntt_split(const bgv_ctx* c, int* p1, int* p2);
// true when the forward NTT has two passes (log N > 8), so the second can be fused
bool ntt_fused_inner_ok(const bgv_ctx* c);
// ModUp output y [n][dn][level+K][N] (coefficient form; the own-digit rows are not
// read): first NTT pass in place, then the second pass fused with the inner product
// -> u [n][2][level+K][N].  The own-digit rows are the rows of x, the switched
// polynomial in evaluation form ([n][level][N] at ciphertext stride x_ct_stride).  With
// dtop, u's top row (row level - 1) of ciphertext ct and component comp receives
// + pmod_top * dtop[ct * dtop_ct + comp * dtop_comp] (evaluation form, pmod_top = P mod
// q_{level-1}).  Rows m >= inv_from (when inv_from >= 0) leave after the first pass of
// their inverse transform; ntt_inverse_last_pass completes it.
void ntt_pass1_key_inner(bgv_ctx* c, uint64_t* y, const uint64_t* x, int64_t x_ct_stride, const uint64_t* key,
                         uint64_t* u, int n, int level, bool pass1_done = false, const uint64_t* dtop = nullptr,
                         int64_t dtop_ct = 0, int64_t dtop_comp = 0, double pmod_top = 0.0, int inv_from = -1);
// true when the fused ModUp below applies (two-pass transforms whose first pass has 5..8
// stages, digits of 1, 2, 4 or 6 primes)
bool modup_cols_ok(const bgv_ctx* c);
// true when the fused ModDown below applies to a batch of n ciphertexts (two-pass transforms
// whose first pass has 5..8 stages, K <= 6, and the setting above)
bool moddown_cols_ok(const bgv_ctx* c, int n);
// From u [n][2][level+K][N], whose top row holds u_top + P d_top and whose top and special
// rows have had the first pass of their inverse transform, the merged ModDown/switch
// correction e [n][2][level-1][N] after the first pass of its forward transform
void moddown_cols(bgv_ctx* c, const uint64_t* u, uint64_t* e, int n, int level, int t_exp);
// From xh [n][level][N] -- x after the first pass of its inverse transform -- the ModUp output
// y [n][dn][level+K][N] with the first forward pass done on every non-own row (as ModUp and
// that pass would leave it); x's own-digit rows are not written
void modup_cols(bgv_ctx* c, const uint64_t* xh, uint64_t* y, int n, int level);
// the first pass of the inverse transform alone, from src into d
void ntt_inverse_first_pass(bgv_ctx* c, uint64_t* d, const uint64_t* src, int n_limbs, LimbMap lm);
// the last pass of the inverse transform alone (two-pass transforms), in place
void ntt_inverse_last_pass(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm);
// the first pass of the forward transform alone, in place
void ntt_forward_first_pass(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm);
// NTT over n_limbs limbs of length N at d (limb l uses the prime given by lm).
// Epilogue of the last forward pass over rows (cc, i), i < rows, of the
// transformed data: with e the transformed value,
//   out = ((a - e * sv_i) + b * sb_i) * qt_i          (mod q_i)
// where a row (cc, i) is at a + cc * a_cc + i * N, b (optional: null) likewise,
// sv null stands for 1, and out has the layout of the data.
struct NttEpi {
  const uint64_t* a;
  int64_t a_cc;
  const uint64_t* b;
  int64_t b_cc;
  const double* sb;
  const double* sv;
  const double* qt;
  uint64_t* out;
  int rows;
};
// the first pass reads src when it is given (out of place), every pass writes d;
// with epi the last forward pass writes epi->out instead (see NttEpi)
void ntt(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm, bool inverse, const uint64_t* src = nullptr,
         const NttEpi* epi = nullptr);
// the last pass of the forward transform alone (two-pass transforms), with the epilogue
void ntt_forward_last_pass(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm, const NttEpi* epi);

// out = a (op) b elementwise per limb; op 0 add, 1 sub; b_bcast: b has one ciphertext
void add_sub(bgv_ctx* c, const uint64_t* a, const uint64_t* b, uint64_t* out, int n, int level, int op, bool b_bcast,
             int sa, int sb);
void negate(bgv_ctx* c, const uint64_t* a, uint64_t* out, int n, int level);
// out = a * s_i per limb (s per prime given as a double table of size level)
void mul_scalar(bgv_ctx* c, const uint64_t* a, uint64_t* out, int n, int level, const double* s_host);
// add s_i to every word of component 0
void add_const(bgv_ctx* c, const uint64_t* a, uint64_t* out, int n, int level, const double* s_host);
// tensor: d01 [n][2][level][N] (d0, d1) and d2 [n][level][N] from a, b [n][2][level][N]
// (sa, sb: limbs per polynomial of a and b in memory when above level; 0: level)
void tensor(bgv_ctx* c, const uint64_t* a, const uint64_t* b, uint64_t* d01, uint64_t* d2, int n, int level,
            bool b_bcast, int sa = 0, int sb = 0);
// Pairs of one multi-pair tensor sum (at most TS_MAX per launch).
constexpr int TS_MAX = 16;
struct TensorPairs {
  const uint64_t* a[TS_MAX];
  const uint64_t* b[TS_MAX];
  int bb[TS_MAX];  // b is one ciphertext broadcast over the batch
  int sa[TS_MAX];  // limbs per polynomial of a and b in memory (at least the level; 0: the level)
  int sb[TS_MAX];
};
// d01, d2 = sum over the np pairs of their tensor products (added to what they hold with acc)
void tensor_sum(bgv_ctx* c, const TensorPairs& tp, int np, uint64_t* d01, uint64_t* d2, int n, int level, bool acc);
// ModUp of the coefficient-form limbs x [n][level][N] -> y [n][dnum'][level+K][N] (coefficient form,
// own-digit rows left untouched)
void mod_up(bgv_ctx* c, const uint64_t* x, uint64_t* y, int n, int level);
// copy the evaluation-form own-digit rows of x (ciphertext b at x + b*x_ct_stride, rows [level][N]) into y
void mod_up_copy_own(bgv_ctx* c, const uint64_t* x_eval, int64_t x_ct_stride, uint64_t* y, int n, int level);
// u [n][2][level+K][N] = sum_j y[n][j][m] * key[j][c][row(m)]
void key_inner(bgv_ctx* c, const uint64_t* y, const uint64_t* key, uint64_t* u, int n, int level);
// delta rows: from the coefficient-form special limbs of polynomial cc (K rows at
// u_coeff + cc * u_stride) write dl [n][2][level][N] (coefficient form) = FBC_{P->Q}([u_P t^-1]_P)
void mod_down_delta(bgv_ctx* c, const uint64_t* u_coeff, int64_t u_stride, uint64_t* dl, int n, int level,
                    int t_exp);
// out[n][2][level] = add[n][c][i] + (u[n][c][i] - t dl[n][c][i]) * P^-1   (evaluation form)
// add points at [n][3][level][N] tensor output (components 0, 1) or [n][2][level][N] with add_stride
void mod_down_final(bgv_ctx* c, const uint64_t* u, const uint64_t* dl, const uint64_t* addsrc,
                    int64_t add_ct_stride, uint64_t* out, int n, int level, int t_exp);
// single drop: w rows from the coefficient-form top limbs top [n][2][N]:
// wrow [n][2][level-1][N] = centered([top t^-1]_{q_top}) mod q_i  (coefficient form)
void msw_w(bgv_ctx* c, const uint64_t* top, uint64_t* wrow, int n, int level, int t_exp);
// (part 2, out_i = (a_i - t w_i) q_top^-1, is the epilogue of the forward NTT of w)
// multi-drop correction: from the dropped limbs tl [n][2][level-to][N] (coefficient form),
// e [n][2][to][N] = t S (coefficient form) with S the combined drop correction; the
// switched limb is (c_i - NTT(e_i)) prod q_dropped^-1 (see kernels.hip)
void msw_corr(bgv_ctx* c, const uint64_t* tl, uint64_t* e, int n, int level, int to, int t_exp);
// Terms and sums of one multi-output linear combination (at most LC_MAXT terms,
// LC_MAXO sums per launch).
constexpr int LC_MAXT = 16;
constexpr int LC_MAXO = 24;
struct LinMulti {
  const uint64_t* x[LC_MAXT];
  int xs[LC_MAXT];  // limbs per polynomial of term t in memory (at least the level; 0: the level)
  uint64_t* out[LC_MAXO];
  int row[LC_MAXO][LC_MAXT];  // coefficient row of term t in sum o; -1: absent
  int cst_row[LC_MAXO];       // row of the constant of sum o; -1: none
};
// scs (optional): the coefficient of every row as a centered integer, |c| < 2^24 (exact
// accumulation of split terms; see kernels.hip); null: residues sc[row][i] only
void lincomb_multi(bgv_ctx* c, const LinMulti& m, int nt, int no, const double* sc, int sc_stride, const double* scs,
                   int n, int level);
// out = sum_t sc[rows[t]][i] * xs[t] (+ sc[cst_row][i] on component 0); nt <= 16 terms, all at `level`
void lincomb(bgv_ctx* c, const uint64_t* const* xs, const int* rows, int nt, const double* sc, int sc_stride,
             int cst_row, uint64_t* out, int n, int level);
// product step with the modulus switch merged into ModDown, part 1 (part 2 is the
// epilogue of the forward NTT of e); dtop null: u's top row already holds u_top + P d_top
void ms_corr(bgv_ctx* c, const uint64_t* up, int64_t up_stride, const uint64_t* utop, int64_t ut_stride,
             const uint64_t* dtop, int64_t dt_stride, uint64_t* e, int n, int level, int t_exp);
// out (one ciphertext) = sum of the n ciphertexts of x
void batch_sum(bgv_ctx* c, const uint64_t* x, uint64_t* out, int n, int level);
// automorphism in evaluation form: for each of n ciphertexts, `rows` limbs at x + ct*xs -> y + ct*ys
void automorph(bgv_ctx* c, const uint64_t* x, int64_t xs, uint64_t* y, int64_t ys, int n, int rows, int g);
// signed small integers (int64 [N] per poly) -> residues [n_polys][rows][N] under primes given by lm
void from_signed(bgv_ctx* c, const int64_t* v, uint64_t* y, int n_polys, int rows, LimbMap lm);
// elementwise: out = a*b (+ sign * c*d) style helpers for encryption / keys
void mul_pointwise(bgv_ctx* c, const uint64_t* a, const uint64_t* b, uint64_t* out, int n_limbs, LimbMap lm,
                   int64_t a_stride_limbs_bcast);
// decrypt phase: v[n][level] = c0 + c1 * S (S [level][N] evaluation form of s)
void phase(bgv_ctx* c, const uint64_t* ct, const uint64_t* S, uint64_t* v, int n, int level);
// encryption: c0 = M - C1*S  with M [n][L][N], C1 [n][L][N], S [L][N]; writes ct [n][2][L][N]
void enc_combine(bgv_ctx* c, const uint64_t* M, const uint64_t* C1, const uint64_t* S, uint64_t* ct, int n);
// key: b = -A*S + t*E + [m in digit j] (P mod q_m) S'
void key_combine(bgv_ctx* c, const uint64_t* A, const uint64_t* S, const uint64_t* E, const uint64_t* Sp,
                 uint64_t* key, int dnum);
}  // namespace lk

bool hip_ok(bgv_ctx* c, hipError_t e, const char* what);

// The allocation-free variant's scratch: the device address of a file-scope device array of
// BGV_NOALLOC_SCRATCH_WORDS words on the current device, looked up once per device and kept
// (kernels.hip).  Returns null if the runtime cannot resolve it.
uint64_t* noalloc_scratch_ptr(int* device);
