// Elementwise and base-conversion kernels of the BGV hot path (gfx950).
//
// Layout of a ciphertext batch: [n][2][level][N] uint64 residues; limb i of a
// component uses prime q_i.  Evaluation-form kernels work word by word; the
// base-conversion kernels (ModUp, ModDown, modulus switching) work on
// coefficient-form limbs produced by the INTT, one coefficient per thread.
#include <mutex>

#include "ctx.hpp"

namespace {

constexpr int BS = 256;

struct Tab64 {
  double v[64];
};

inline dim3 grid_for(int N, int y, int z = 1) { return dim3(N >= BS ? N / BS : 1, y, z); }
inline int block_for(int N) { return N >= BS ? BS : N; }

// a and b may be views of the lower `level` limbs of deeper batches: sa / sb limbs per
// polynomial in memory (the output is contiguous)
__global__ void k_add_sub(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b, uint64_t* __restrict__ out,
                          int level, int N, int op, int b_bcast, int sa, int sb, const PrimeD* __restrict__ pc) {
  const int limb = blockIdx.y;
  const int poly = limb / level, pi = limb - poly * level;
  const double q = pc[pi].q;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t ia = ((size_t)poly * sa + pi) * N + n0;
  const size_t ib = ((size_t)(b_bcast ? poly % 2 : poly) * sb + pi) * N + n0;
  double x = u2d(a[ia]), y = u2d(b[ib]);
  double r = op == 0 ? x + y : x - y;
  r = r >= q ? r - q : r;
  r = r < 0.0 ? r + q : r;
  out[(size_t)limb * N + n0] = d2u(r);
}

__global__ void k_negate(const uint64_t* __restrict__ a, uint64_t* __restrict__ out, int level, int N,
                         const PrimeD* __restrict__ pc) {
  const int limb = blockIdx.y;
  const double q = pc[limb % level].q;
  const size_t i = (size_t)limb * N + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double x = u2d(a[i]);
  out[i] = d2u(x == 0.0 ? 0.0 : q - x);
}

__global__ void k_mul_scalar(const uint64_t* __restrict__ a, uint64_t* __restrict__ out, int level, int N, Tab64 s,
                             const PrimeD* __restrict__ pc) {
  const int limb = blockIdx.y;
  const int pi = limb % level;
  const double q = pc[pi].q, qinv = pc[pi].qinv;
  const size_t i = (size_t)limb * N + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  out[i] = d2u(canon(mul_lazy(u2d(a[i]), s.v[pi], q, qinv), q));
}

__global__ void k_add_const(const uint64_t* __restrict__ a, uint64_t* __restrict__ out, int level, int N, Tab64 s,
                            const PrimeD* __restrict__ pc) {
  const int limb = blockIdx.y;
  const int pi = limb % level;
  const int comp = (limb / level) & 1;
  const double q = pc[pi].q;
  const size_t i = (size_t)limb * N + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double x = u2d(a[i]);
  if (comp == 0) {
    x += s.v[pi];
    x = x >= q ? x - q : x;
  }
  out[i] = d2u(x);
}

// d01[b][0] = a0 b0, d01[b][1] = a0 b1 + a1 b0, d2[b] = a1 b1
// Tensor product (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1).
__global__ void k_tensor(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b, uint64_t* __restrict__ d,
                         uint64_t* __restrict__ d2, int level, int N, int b_bcast, int sa, int sb,
                         const PrimeD* __restrict__ pc) {
  const int ct = blockIdx.y / level;
  const int i = blockIdx.y % level;
  const double q = pc[i].q, qinv = pc[i].qinv;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t L2 = (size_t)level * N;
  const size_t LA = (size_t)sa * N, LB = (size_t)sb * N;  // polynomial strides of the operands
  const uint64_t* A = a + (size_t)ct * 2 * LA + (size_t)i * N + n0;
  const uint64_t* B = b + (size_t)(b_bcast ? 0 : ct) * 2 * LB + (size_t)i * N + n0;
  uint64_t* D = d + (size_t)ct * 2 * L2 + (size_t)i * N + n0;
  // a is read once; a broadcast b is shared by every ciphertext and stays cached
  const double a0 = u2d(ld_once(A)), a1 = u2d(ld_once(A + LA));
  const double b0 = u2d(b_bcast ? B[0] : ld_once(B)), b1 = u2d(b_bcast ? B[LB] : ld_once(B + LB));
  uint64_t* E = d2 + (size_t)ct * L2 + (size_t)i * N + n0;
  const double v0 = mul_lazy(a0, b0, q, qinv);
  const double v1 = mul_lazy(a0, b1, q, qinv) + mul_lazy(a1, b0, q, qinv);
  const double v2 = mul_lazy(a1, b1, q, qinv);
  D[0] = d2u(canon(red(v0, q, qinv), q));
  D[L2] = d2u(canon(red(v1, q, qinv), q));
  E[0] = d2u(canon(red(v2, q, qinv), q));
}

// Sum of the tensor products of np pairs in one pass: (d0, d1, d2) = sum_t (a0 b0, a0 b1 +
// a1 b0, a1 b1) of pair t (b broadcast over the batch where bb[t]); with acc the sum is added
// to what d and d2 hold.  Each operand is read once.
__global__ void k_tensor_sum(lk::TensorPairs tp, int np, uint64_t* __restrict__ d, uint64_t* __restrict__ d2,
                             int level, int N, int acc, const PrimeD* __restrict__ pc) {
  const int ct = blockIdx.y / level;
  const int i = blockIdx.y % level;
  const double q = pc[i].q, qinv = pc[i].qinv;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t L2 = (size_t)level * N;
  const size_t off = (size_t)i * N + n0;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int t = 0; t < np; ++t) {
    const size_t LA = (size_t)(tp.sa[t] ? tp.sa[t] : level) * N;  // polynomial strides (0: level)
    const size_t LB = (size_t)(tp.sb[t] ? tp.sb[t] : level) * N;
    const uint64_t* A = tp.a[t] + (size_t)ct * 2 * LA + off;
    const uint64_t* B = tp.b[t] + (size_t)(tp.bb[t] ? 0 : ct) * 2 * LB + off;
    const double a0 = u2d(ld_once(A)), a1 = u2d(ld_once(A + LA));
    const double b0 = u2d(tp.bb[t] ? B[0] : ld_once(B)), b1 = u2d(tp.bb[t] ? B[LB] : ld_once(B + LB));
    v0 = red(v0 + mul_lazy(a0, b0, q, qinv), q, qinv);
    v1 = red(v1 + mul_lazy(a0, b1, q, qinv) + mul_lazy(a1, b0, q, qinv), q, qinv);
    v2 = red(v2 + mul_lazy(a1, b1, q, qinv), q, qinv);
  }
  uint64_t* D = d + (size_t)ct * 2 * L2 + off;
  uint64_t* E = d2 + (size_t)ct * L2 + off;
  if (acc) {
    v0 += u2d(D[0]);
    v1 += u2d(D[L2]);
    v2 += u2d(E[0]);
  }
  D[0] = d2u(canon(red(v0, q, qinv), q));
  D[L2] = d2u(canon(red(v1, q, qinv), q));
  E[0] = d2u(canon(red(v2, q, qinv), q));
}

// ModUp: x [n][level][N] coefficient form -> y [n][dn][level+K][N].  For digit j
// with primes D_j: v_i = [x_i Qhat_i^-1]_{q_i} (in [0, q_i)), and for every target
// prime m outside D_j: y_m = sum_i v_i (Qhat_i mod m) mod m.
__global__ void k_mod_up(const uint64_t* __restrict__ x, uint64_t* __restrict__ y, int level, int N, int alpha,
                         int dn, int K, int Lfull, int Ltot, const double* __restrict__ tab, size_t tab_stride_lvl,
                         size_t tab_stride_dig, const PrimeD* __restrict__ pc) {
  const int ct = blockIdx.y / dn;
  const int j = blockIdx.y % dn;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lo = j * alpha;
  const int hi = min(lo + alpha, level);
  const int na = hi - lo;
  const double* inv = tab + (size_t)level * tab_stride_lvl + (size_t)j * tab_stride_dig;
  const double* basis = inv + alpha;
  const uint64_t* X = x + (size_t)ct * level * N + n0;
  double v[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (a < na) {
      const int i = lo + a;
      const double q = pc[i].q, qinv = pc[i].qinv;
      v[a] = canon(mul_lazy(u2d(ld_once(X + (size_t)i * N)), inv[a], q, qinv), q);
    } else {
      v[a] = 0.0;
    }
  }
  const int rows = level + K;
  uint64_t* Y = y + ((size_t)ct * dn + j) * rows * N + n0;
  for (int m = 0; m < rows; ++m) {
    if (m >= lo && m < hi) continue;
    const int pm = m < level ? m : Lfull + (m - level);
    const double q = pc[pm].q, qinv = pc[pm].qinv;
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (a < na) acc += mul_lazy(v[a], basis[(size_t)a * Ltot + pm], q, qinv);
    }
    Y[(size_t)m * N] = to_u(acc, q, qinv);
  }
}

// y[ct][j][m] = x_eval[ct][m] for the primes m of digit j
__global__ void k_mod_up_copy_own(const uint64_t* __restrict__ x, int64_t x_ct_stride, uint64_t* __restrict__ y,
                                  int level, int N, int alpha, int dn, int K) {
  const int ct = blockIdx.y / dn;
  const int j = blockIdx.y % dn;
  const int lo = j * alpha;
  const int hi = min(lo + alpha, level);
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int rows = level + K;
  for (int m = lo; m < hi; ++m)
    y[(((size_t)ct * dn + j) * rows + m) * N + n0] = x[(size_t)ct * x_ct_stride + (size_t)m * N + n0];
}

// u[ct][c][m] = sum_j y[ct][j][m] * key[j][c][row(m)]  (evaluation form).
// CB ciphertexts per thread share each key word.
template <int CB>
__global__ void k_key_inner(const uint64_t* __restrict__ y, const uint64_t* __restrict__ key, uint64_t* __restrict__ u,
                            int level, int N, int dn, int K, int Lfull, int Ltot, int n_ct,
                            const PrimeD* __restrict__ pc) {
  const int m = blockIdx.y;
  const int rows = level + K;
  const int pm = m < level ? m : Lfull + (m - level);
  const double q = pc[pm].q, qinv = pc[pm].qinv;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ct0 = blockIdx.z * CB;
  double acc0[CB], acc1[CB];
#pragma unroll
  for (int b = 0; b < CB; ++b) acc0[b] = acc1[b] = 0.0;
  for (int j = 0; j < dn; ++j) {
    const double kb = u2d(key[(((size_t)j * 2 + 0) * Ltot + pm) * N + n0]);
    const double ka = u2d(key[(((size_t)j * 2 + 1) * Ltot + pm) * N + n0]);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      if (ct0 + b < n_ct) {
        const double yy = u2d(y[(((size_t)(ct0 + b) * dn + j) * rows + m) * N + n0]);
        acc0[b] += mul_lazy(yy, kb, q, qinv);
        acc1[b] += mul_lazy(yy, ka, q, qinv);
        if ((j & 3) == 3) {
          acc0[b] = red(acc0[b], q, qinv);
          acc1[b] = red(acc1[b], q, qinv);
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    if (ct0 + b < n_ct) {
      uint64_t* U = u + ((size_t)(ct0 + b) * 2 * rows + m) * N + n0;
      U[0] = to_u(acc0[b], q, qinv);
      U[(size_t)rows * N] = to_u(acc1[b], q, qinv);
    }
  }
}

// ModDown correction: from the coefficient-form special rows of polynomial cc (K rows
// at u + cc * u_stride, N words apart), w_k = [u_k t^-1]_{p_k}, v_k = [w_k Phat_k^-1]_{p_k}
// (both in [0, p_k)), dl_i = sum_k v_k (Phat_k mod q_i) mod q_i.
__global__ void k_mod_down_delta(const uint64_t* __restrict__ u, int64_t u_stride, uint64_t* __restrict__ dl,
                                 int level, int N, int K,
                                 int Lfull, const double* __restrict__ md, const double* __restrict__ tinv,
                                 const PrimeD* __restrict__ pc) {
  const int cc = blockIdx.y;  // ct * 2 + comp
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t* U = u + (size_t)cc * u_stride + n0;
  const double* phat_inv = md;
  const double* phat_mod = md + K;  // [K][Lfull]
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < K) {
      const int pk = Lfull + k;
      const double q = pc[pk].q, qinv = pc[pk].qinv;
      const double w = canon(mul_lazy(u2d(U[(size_t)k * N]), tinv[pk], q, qinv), q);
      v[k] = canon(mul_lazy(w, phat_inv[k], q, qinv), q);
    } else {
      v[k] = 0.0;
    }
  }
  uint64_t* D = dl + (size_t)cc * level * N + n0;
  for (int i = 0; i < level; ++i) {
    const double q = pc[i].q, qinv = pc[i].qinv;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k < K) acc += mul_lazy(v[k], phat_mod[(size_t)k * Lfull + i], q, qinv);
    }
    D[(size_t)i * N] = to_u(acc, q, qinv);
  }
}

// out[ct][c][i] = add[ct][c][i] + (u[ct][c][i] - t dl[ct][c][i]) P^-1  (evaluation form);
// components c >= add_comps get no addend.
__global__ void k_mod_down_final(const uint64_t* __restrict__ u, const uint64_t* __restrict__ dl,
                                 const uint64_t* __restrict__ add, int64_t add_ct_stride, int add_comps,
                                 uint64_t* __restrict__ out, int level, int N, int K, const double* __restrict__ pinv,
                                 const double* __restrict__ tmod, const PrimeD* __restrict__ pc) {
  const int i = blockIdx.y % level;
  const int cc = blockIdx.y / level;  // ct * 2 + comp
  const int ct = cc >> 1, comp = cc & 1;
  const int rows = level + K;
  const double q = pc[i].q, qinv = pc[i].qinv;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double uu = u2d(u[((size_t)cc * rows + i) * N + n0]);
  const double dd = u2d(dl[((size_t)cc * level + i) * N + n0]);
  const double diff = uu - mul_lazy(dd, tmod[i], q, qinv);  // |.| < 2q
  double r = mul_lazy(red(diff, q, qinv), pinv[i], q, qinv);
  if (comp < add_comps) r += u2d(add[(size_t)ct * add_ct_stride + ((size_t)comp * level + i) * N + n0]);
  out[((size_t)cc * level + i) * N + n0] = to_u(r, q, qinv);
}

// single modulus switch, part 1: top [n*2][N] coefficient form -> w rows [n*2][level-1][N]
__global__ void k_msw_w(const uint64_t* __restrict__ top, uint64_t* __restrict__ w, int level, int N,
                        double tinv_top, const PrimeD* __restrict__ pc) {
  const int cc = blockIdx.y;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int it = level - 1;
  const double qt = pc[it].q, qtinv = pc[it].qinv;
  double wt = canon(mul_lazy(u2d(top[(size_t)cc * N + n0]), tinv_top, qt, qtinv), qt);
  const double half = (qt - 1.0) * 0.5;
  wt = wt > half ? wt - qt : wt;  // centered, |wt| < 2^49 <= every q_i
  uint64_t* W = w + (size_t)cc * (level - 1) * N + n0;
  for (int i = 0; i < level - 1; ++i) {
    const double q = pc[i].q;
    W[(size_t)i * N] = d2u(wt < 0.0 ? wt + q : wt);
  }
}

// at most MSW_MAXD drops per launch of the repeated switch (longer chains are chained steps)
constexpr int MSW_MAXD = 16;

// Repeated modulus switch in correction form.  tl [n*2][nd][N] holds the nd = level - to
// dropped limbs of every polynomial in coefficient form (limb to + k at row k).  The w of
// every single drop is formed top down: the current value of the limb about to be dropped
// is its input transformed by every drop above it.  The nd sequential drops then
// amount to c_i -> (c_i - t S) prod_e q_e^-1 with S = w_0 + q_0 (w_1 + q_1 (w_2 + ...)), q_e
// the e-th prime dropped.  e_i = t S mod q_i (coefficient form) is written for i < to; the
// caller transforms it and applies (c_i - e_i) prod_e q_e^-1 in evaluation form.  The chain
// is descending, so every dropped prime is below q_i and q_e mod q_i = q_e.
__global__ void k_msw_corr(const uint64_t* __restrict__ tl, uint64_t* __restrict__ e, int level, int to, int N,
                           const double* __restrict__ msw, int L, const double* __restrict__ tinv,
                           const double* __restrict__ tmod, const PrimeD* __restrict__ pc) {
  const int cc = blockIdx.y;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nd = level - to;
  const uint64_t* X = tl + (size_t)cc * nd * N + n0;
  double wv[MSW_MAXD];
#pragma unroll
  for (int d = 0; d < MSW_MAXD; ++d) {
    wv[d] = 0.0;
    if (d < nd) {
      const int top = level - 1 - d;
      const double q = pc[top].q, qinv = pc[top].qinv;
      double cur = u2d(ld_once(X + (size_t)(top - to) * N));
#pragma unroll
      for (int f = 0; f < d; ++f) {
        const int up = level - 1 - f;
        const double diff = cur - mul_lazy(wv[f] < 0.0 ? wv[f] + q : wv[f], tmod[top], q, qinv);
        cur = mul_lazy(red(diff, q, qinv), msw[(size_t)up * L + top], q, qinv);
      }
      double wt = canon(mul_lazy(canon(red(cur, q, qinv), q), tinv[top], q, qinv), q);
      const double half = (q - 1.0) * 0.5;
      wv[d] = wt > half ? wt - q : wt;
    }
  }
  uint64_t* E = e + (size_t)cc * to * N + n0;
  for (int i = 0; i < to; ++i) {
    const double q = pc[i].q, qinv = pc[i].qinv;
    double acc = 0.0;
#pragma unroll
    for (int d = MSW_MAXD - 1; d >= 0; --d) {
      if (d < nd) {
        const double qd = pc[level - 1 - d].q;  // below q_i
        acc = red(wv[d] + mul_lazy(acc, qd, q, qinv), q, qinv);
      }
    }
    E[(size_t)i * N] = to_u(mul_lazy(acc, tmod[i], q, qinv), q, qinv);
  }
}

// out[c][i] = sum over the batch of in[b][c][i]  (one block row per limb of one ciphertext)
__global__ void k_batch_sum(const uint64_t* __restrict__ x, uint64_t* __restrict__ out, int n, int level, int N,
                            const PrimeD* __restrict__ pc) {
  const int limb = blockIdx.y;  // comp * level + i
  const int i = limb % level;
  const double q = pc[i].q, qinv = pc[i].qinv;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)2 * level * N;
  double acc = 0.0;
  for (int b = 0; b < n; ++b) {
    acc += u2d(x[(size_t)b * stride + (size_t)limb * N + n0]);
    if ((b & 3) == 3) acc = red(acc, q, qinv);
  }
  out[(size_t)limb * N + n0] = to_u(acc, q, qinv);
}

// out[ct][c][i] = sum_t sc[row_t][i] * x_t[ct][c][i] (+ sc[cst_row][i] on component 0): the inner
// sums of the polynomial evaluator in one pass (every term at the same level).
struct LinTerms {
  const uint64_t* x[16];
  int row[16];
};

__global__ void k_lincomb(LinTerms terms, int nt, const double* __restrict__ sc, int sc_stride, int cst_row,
                          uint64_t* __restrict__ out, int level, int N, const PrimeD* __restrict__ pc) {
  const int limb = blockIdx.y;
  const int i = limb % level;
  const int comp = (limb / level) & 1;
  const double q = pc[i].q, qinv = pc[i].qinv;
  const size_t off = (size_t)limb * N + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  for (int t = 0; t < nt; ++t) {
    acc += mul_lazy(u2d(terms.x[t][off]), sc[(size_t)terms.row[t] * sc_stride + i], q, qinv);
    if ((t & 3) == 3) acc = red(acc, q, qinv);
  }
  if (comp == 0 && cst_row >= 0) acc += sc[(size_t)cst_row * sc_stride + i];
  out[off] = to_u(acc, q, qinv);
}

// Several inner sums over one set of terms in one pass: out_o[ct][c][i] =
// sum_t c_ot x_t[ct][c][i] (+ the constant sc[cst_row[o]][i] on component 0), where
// c_ot is the coefficient of row row[o][t] (-1: the term is absent from sum o).  Each
// term is read once for all sums, and the block's coefficient matrix is staged in LDS
// first.  With SPLIT the coefficients come as centered integers scs[row], |c| < 2^24:
// every term is split into 25-bit halves, so that each product is below 2^49 and the
// sums of at most 16 of them are exact in binary64; a sum then takes one modular
// product (hi 2^25 + lo) instead of one per term.  Without SPLIT the coefficients are
// residues sc[row][i] and every product is reduced.
template <bool SPLIT>
__global__ void k_lincomb_multi(lk::LinMulti m, int nt, int no, const double* __restrict__ sc, int sc_stride,
                                const double* __restrict__ scs, int level, int N, const PrimeD* __restrict__ pc) {
  constexpr int T = lk::LC_MAXT;
  __shared__ double cf[lk::LC_MAXO * T];
  const int limb = blockIdx.y;
  const int i = limb % level;
  const int comp = (limb / level) & 1;
  for (int k = threadIdx.x; k < no * T; k += blockDim.x) {
    const int o = k / T, t = k % T;
    const int row = t < nt ? m.row[o][t] : -1;
    cf[k] = row < 0 ? 0.0 : (SPLIT ? scs[row] : sc[(size_t)row * sc_stride + i]);
  }
  __syncthreads();
  const double q = pc[i].q, qinv = pc[i].qinv;
  const size_t pos = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t off = (size_t)limb * N + pos;
  const int poly = limb / level;  // ciphertext * 2 + component
  // term t's word: its polynomial stride is xs[t] limbs (at least the level; 0: the level)
  auto xoff = [&](int t) { return ((size_t)poly * (m.xs[t] ? m.xs[t] : level) + i) * N + pos; };
  if constexpr (SPLIT) {
    double xh[T], xl[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const uint64_t v = t < nt ? ld_once(m.x[t] + xoff(t)) : 0;
      xh[t] = split_hi(v);
      xl[t] = split_lo(v);
    }
    for (int o = 0; o < no; ++o) {
      double hi = 0.0, lo = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        if (t < nt) {
          const double c = cf[o * T + t];
          hi = __builtin_fma(c, xh[t], hi);
          lo = __builtin_fma(c, xl[t], lo);
        }
      }
      double acc = split_combine(hi, lo, q, qinv);
      if (comp == 0 && m.cst_row[o] >= 0) acc += sc[(size_t)m.cst_row[o] * sc_stride + i];
      __builtin_nontemporal_store(to_u(acc, q, qinv), m.out[o] + off);
    }
  } else {
    double x[T];
#pragma unroll
    for (int t = 0; t < T; ++t) x[t] = t < nt ? u2d(ld_once(m.x[t] + xoff(t))) : 0.0;
    for (int o = 0; o < no; ++o) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        if (t < nt) {
          acc += mul_lazy(x[t], cf[o * T + t], q, qinv);
          if ((t & 3) == 3) acc = red(acc, q, qinv);
        }
      }
      if (comp == 0 && m.cst_row[o] >= 0) acc += sc[(size_t)m.cst_row[o] * sc_stride + i];
      __builtin_nontemporal_store(to_u(acc, q, qinv), m.out[o] + off);
    }
  }
}

// Product step with the modulus switch merged into ModDown, part 1 (coefficient form).
// For polynomial cc = ct*2+c: from its coefficient-form special rows (K rows at
// up + cc * up_stride, N words apart) the ModDown correction
// wt_i = FBC_{P->Q}([u_P t^-1]_P) is formed for every q_i; the top
// limb of the relinearised product in coefficient form is
//   o_top = d_top + (u_top - t wt_top) P^-1,
// its switch correction w = centered([o_top t^-1]_{q_top}), and the combined
// correction e_i = t P^-1 wt_i + t w (mod q_i) for i < level-1 is written to e.
// u_top and d_top of polynomial cc (coefficient form) are at utop + cc * ut_stride and
// dtop + cc * dt_stride.
__global__ void k_ms_corr(const uint64_t* __restrict__ up, int64_t up_stride, const uint64_t* __restrict__ utop,
                          int64_t ut_stride, const uint64_t* __restrict__ dtop, int64_t dt_stride,
                          uint64_t* __restrict__ e, int level, int N, int K, int Lfull,
                          const double* __restrict__ md, const double* __restrict__ mdfold,
                          const double* __restrict__ tinv, const double* __restrict__ tmod,
                          const PrimeD* __restrict__ pc) {
  const int cc = blockIdx.y;  // ct * 2 + comp
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double* phat_inv = md;
  const double* phat_mod = md + K;
  const double* pinv = md + K + (size_t)K * Lfull;
  const uint64_t* U = up + (size_t)cc * up_stride + n0;
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < K) {
      const int pk = Lfull + k;
      const double q = pc[pk].q, qinv = pc[pk].qinv;
      const double w = canon(mul_lazy(u2d(ld_once(U + (size_t)k * N)), tinv[pk], q, qinv), q);
      v[k] = canon(mul_lazy(w, phat_inv[k], q, qinv), q);
    } else {
      v[k] = 0.0;
    }
  }
  auto fbc = [&](int i, double q, double qinv) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < K) acc += mul_lazy(v[k], phat_mod[(size_t)k * Lfull + i], q, qinv);
    return canon(red(acc, q, qinv), q);
  };
  const int it = level - 1;
  double wms;
  {
    const double q = pc[it].q, qinv = pc[it].qinv;
    const double wt = fbc(it, q, qinv);
    const double ut = u2d(ld_once(utop + (size_t)cc * ut_stride + n0));
    // with dtop null, u's top row holds u_top + P d_top: (u_top + P d_top - t wt) P^-1 is
    // the same residue as d_top + (u_top - t wt) P^-1
    const double dt = dtop ? u2d(ld_once(dtop + (size_t)cc * dt_stride + n0)) : 0.0;
    const double diff = red(ut - mul_lazy(wt, tmod[it], q, qinv), q, qinv);
    const double o = canon(red(dt + mul_lazy(diff, pinv[it], q, qinv), q, qinv), q);
    const double w = canon(mul_lazy(o, tinv[it], q, qinv), q);
    wms = w > (q - 1.0) * 0.5 ? w - q : w;  // centered
  }
  // e_i = t P^-1 wt_i + t w with t P^-1 folded into the conversion constants
  // (mdfold[k][i] = Phat_k t P^-1 mod q_i): K + 1 products per word; |a| < K q <= 8 q
  uint64_t* E = e + (size_t)cc * (level - 1) * N + n0;
  for (int i = 0; i < level - 1; ++i) {
    const double q = pc[i].q, qinv = pc[i].qinv;
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < K) a += mul_lazy(v[k], mdfold[(size_t)k * Lfull + i], q, qinv);
    const double b = mul_lazy(wms < 0.0 ? wms + q : wms, tmod[i], q, qinv);
    E[(size_t)i * N] = to_u(red(a, q, qinv) + b, q, qinv);
  }
}

__device__ __forceinline__ uint32_t brv32(uint32_t v, int bits) { return __brev(v) >> (32 - bits); }

// X -> X^g in evaluation form: slot j holds a(psi^(2 brv(j)+1)); the image holds
// a(psi^((2 brv(j)+1) g)), i.e. the input slot j' with 2 brv(j')+1 = (2 brv(j)+1) g mod 2N.
__device__ __forceinline__ uint32_t automorph_src(uint32_t j, int logN, uint32_t g) {
  const uint32_t e = 2 * brv32(j, logN) + 1;
  const uint32_t e2 = (uint32_t)(((uint64_t)e * g) & ((2u << logN) - 1));
  return brv32((e2 - 1) >> 1, logN);
}

// Multiplying by the odd g mod 2N maps the low bits of an exponent to low bits only, and the
// low bits of 2 brv(j)+1 are the high bits of j: the 2^logB destination slots that share their
// high bits read 2^logB source slots that share theirs.  A block stages that source block in
// LDS (coalesced reads), gathers there and writes its destination block (coalesced writes).
// x and y must not overlap.
__global__ void k_automorph(const uint64_t* __restrict__ x, int64_t xs, uint64_t* __restrict__ y, int64_t ys, int rows,
                            int logN, int logB, uint32_t g) {
  extern __shared__ uint64_t sblk[];
  const int N = 1 << logN, B = 1 << logB;
  const int ct = blockIdx.y / rows;
  const int r = blockIdx.y % rows;
  const uint32_t d0 = (uint32_t)blockIdx.x << logB;  // first destination slot of the block
  const uint32_t s0 = automorph_src(d0, logN, g) & ~(uint32_t)(B - 1);  // its source block
  const uint64_t* __restrict__ xr = x + (size_t)ct * xs + (size_t)r * N + s0;
  for (int t = threadIdx.x; t < B; t += blockDim.x) sblk[t] = __builtin_nontemporal_load(&xr[t]);
  __syncthreads();
  uint64_t* __restrict__ yr = y + (size_t)ct * ys + (size_t)r * N + d0;
  for (int t = threadIdx.x; t < B; t += blockDim.x) yr[t] = sblk[automorph_src(d0 + t, logN, g) - s0];
}

__global__ void k_from_signed(const int64_t* __restrict__ v, uint64_t* __restrict__ y, int rows, int N, LimbMap lm,
                              const PrimeD* __restrict__ pc) {
  const int b = blockIdx.y / rows;
  const int r = blockIdx.y % rows;
  const int pi = limb_prime(lm, r);
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double q = pc[pi].q, qinv = pc[pi].qinv;
  const int64_t s = v[(size_t)b * N + n0];
  // small integers (|s| < 2^52) are exact as doubles
  y[((size_t)b * rows + r) * N + n0] = to_u((double)s, q, qinv);
}

__global__ void k_phase(const uint64_t* __restrict__ ct, const uint64_t* __restrict__ S, uint64_t* __restrict__ v,
                        int level, int N, const PrimeD* __restrict__ pc) {
  const int i = blockIdx.y % level;
  const int b = blockIdx.y / level;
  const double q = pc[i].q, qinv = pc[i].qinv;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t* C = ct + (size_t)b * 2 * level * N + (size_t)i * N + n0;
  const double c0 = u2d(C[0]), c1 = u2d(C[(size_t)level * N]);
  const double s = u2d(S[(size_t)i * N + n0]);
  v[((size_t)b * level + i) * N + n0] = to_u(c0 + mul_lazy(c1, s, q, qinv), q, qinv);
}

// ct[b] = (M[b] - C1[b] S, C1[b]) over L primes
__global__ void k_enc_combine(const uint64_t* __restrict__ M, const uint64_t* __restrict__ C1,
                              const uint64_t* __restrict__ S, uint64_t* __restrict__ ct, int L, int N,
                              const PrimeD* __restrict__ pc) {
  const int i = blockIdx.y % L;
  const int b = blockIdx.y / L;
  const double q = pc[i].q, qinv = pc[i].qinv;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double m = u2d(M[((size_t)b * L + i) * N + n0]);
  const uint64_t c1w = C1[((size_t)b * L + i) * N + n0];
  const double s = u2d(S[(size_t)i * N + n0]);
  uint64_t* out = ct + (size_t)b * 2 * L * N + (size_t)i * N + n0;
  out[0] = to_u(m - mul_lazy(u2d(c1w), s, q, qinv), q, qinv);
  out[(size_t)L * N] = c1w;
}

// key[j][0][m] = -A[j][m] S[m] + t E[j][m] + [m in digit j] (P mod q_m) Sp[m];  key[j][1][m] = A[j][m]
__global__ void k_key_combine(const uint64_t* __restrict__ A, const uint64_t* __restrict__ S,
                              const uint64_t* __restrict__ E, const uint64_t* __restrict__ Sp,
                              uint64_t* __restrict__ key, int Ltot, int L, int N, int alpha, double tfull_unused,
                              const double* __restrict__ tmod_full, const double* __restrict__ pmod,
                              const PrimeD* __restrict__ pc) {
  const int m = blockIdx.y % Ltot;
  const int j = blockIdx.y / Ltot;
  const double q = pc[m].q, qinv = pc[m].qinv;
  const size_t n0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t off = ((size_t)j * Ltot + m) * N + n0;
  const double a = u2d(A[off]);
  const double s = u2d(S[(size_t)m * N + n0]);
  const double e = u2d(E[off]);
  double r = mul_lazy(e, tmod_full[m], q, qinv) - mul_lazy(a, s, q, qinv);
  if (m < L && m / alpha == j) r += mul_lazy(u2d(Sp[(size_t)m * N + n0]), pmod[m], q, qinv);
  key[(((size_t)j * 2 + 0) * Ltot + m) * N + n0] = to_u(r, q, qinv);
  key[(((size_t)j * 2 + 1) * Ltot + m) * N + n0] = A[off];
  (void)tfull_unused;
}

__global__ void k_mul_pointwise(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                uint64_t* __restrict__ out, int N, LimbMap lm, const PrimeD* __restrict__ pc) {
  const int limb = blockIdx.y;
  const int pi = limb_prime(lm, limb);
  const double q = pc[pi].q, qinv = pc[pi].qinv;
  const size_t i = (size_t)limb * N + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  out[i] = d2u(canon(mul_lazy(u2d(a[i]), u2d(b[i]), q, qinv), q));
}

}  // namespace

namespace lk {

void add_sub(bgv_ctx* c, const uint64_t* a, const uint64_t* b, uint64_t* out, int n, int level, int op, bool bb, int sa,
             int sb) {
  hipLaunchKernelGGL(k_add_sub, grid_for(c->N, n * 2 * level), dim3(block_for(c->N)), 0, c->stream, a, b, out, level,
                     c->N, op, bb ? 1 : 0, sa, sb, c->d_prime);
}

void negate(bgv_ctx* c, const uint64_t* a, uint64_t* out, int n, int level) {
  hipLaunchKernelGGL(k_negate, grid_for(c->N, n * 2 * level), dim3(block_for(c->N)), 0, c->stream, a, out, level, c->N,
                     c->d_prime);
}

void mul_scalar(bgv_ctx* c, const uint64_t* a, uint64_t* out, int n, int level, const double* s) {
  Tab64 t;
  for (int i = 0; i < 64; ++i) t.v[i] = i < level ? s[i] : 0.0;
  hipLaunchKernelGGL(k_mul_scalar, grid_for(c->N, n * 2 * level), dim3(block_for(c->N)), 0, c->stream, a, out, level,
                     c->N, t, c->d_prime);
}

void add_const(bgv_ctx* c, const uint64_t* a, uint64_t* out, int n, int level, const double* s) {
  Tab64 t;
  for (int i = 0; i < 64; ++i) t.v[i] = i < level ? s[i] : 0.0;
  hipLaunchKernelGGL(k_add_const, grid_for(c->N, n * 2 * level), dim3(block_for(c->N)), 0, c->stream, a, out, level,
                     c->N, t, c->d_prime);
}

void tensor(bgv_ctx* c, const uint64_t* a, const uint64_t* b, uint64_t* d, uint64_t* d2, int n, int level, bool bb,
            int sa, int sb) {
  hipLaunchKernelGGL(k_tensor, grid_for(c->N, n * level), dim3(block_for(c->N)), 0, c->stream, a, b, d, d2, level,
                     c->N, bb ? 1 : 0, sa ? sa : level, sb ? sb : level, c->d_prime);
}

void tensor_sum(bgv_ctx* c, const TensorPairs& tp, int np, uint64_t* d, uint64_t* d2, int n, int level, bool acc) {
  hipLaunchKernelGGL(k_tensor_sum, grid_for(c->N, n * level), dim3(block_for(c->N)), 0, c->stream, tp, np, d, d2, level,
                     c->N, acc ? 1 : 0, c->d_prime);
}

void mod_up(bgv_ctx* c, const uint64_t* x, uint64_t* y, int n, int level) {
  const int dn = (level + c->alpha - 1) / c->alpha;
  const size_t s_dig = (size_t)c->alpha * (1 + c->Ltot);
  const size_t s_lvl = (size_t)c->dnum * s_dig;
  hipLaunchKernelGGL(k_mod_up, grid_for(c->N, n * dn), dim3(block_for(c->N)), 0, c->stream, x, y, level, c->N,
                     c->alpha, dn, c->prm.K, c->prm.L, c->Ltot, c->d_modup, s_lvl, s_dig, c->d_prime);
}

void mod_up_copy_own(bgv_ctx* c, const uint64_t* x, int64_t x_ct_stride, uint64_t* y, int n, int level) {
  const int dn = (level + c->alpha - 1) / c->alpha;
  hipLaunchKernelGGL(k_mod_up_copy_own, grid_for(c->N, n * dn), dim3(block_for(c->N)), 0, c->stream, x, x_ct_stride, y,
                     level, c->N, c->alpha, dn, c->prm.K);
}

void key_inner(bgv_ctx* c, const uint64_t* y, const uint64_t* key, uint64_t* u, int n, int level) {
  const int dn = (level + c->alpha - 1) / c->alpha;
  const int rows = level + c->prm.K;
  int cb = n >= 4 ? 4 : (n >= 2 ? 2 : 1);
  dim3 grid = grid_for(c->N, rows, (n + cb - 1) / cb);
  dim3 blk(block_for(c->N));
  if (cb == 4)
    hipLaunchKernelGGL((k_key_inner<4>), grid, blk, 0, c->stream, y, key, u, level, c->N, dn, c->prm.K, c->prm.L,
                       c->Ltot, n, c->d_prime);
  else if (cb == 2)
    hipLaunchKernelGGL((k_key_inner<2>), grid, blk, 0, c->stream, y, key, u, level, c->N, dn, c->prm.K, c->prm.L,
                       c->Ltot, n, c->d_prime);
  else
    hipLaunchKernelGGL((k_key_inner<1>), grid, blk, 0, c->stream, y, key, u, level, c->N, dn, c->prm.K, c->prm.L,
                       c->Ltot, n, c->d_prime);
}

void mod_down_delta(bgv_ctx* c, const uint64_t* u, int64_t u_stride, uint64_t* dl, int n, int level, int t_exp) {
  hipLaunchKernelGGL(k_mod_down_delta, grid_for(c->N, n * 2), dim3(block_for(c->N)), 0, c->stream, u, u_stride, dl,
                     level, c->N, c->prm.K, c->prm.L, c->d_moddown, c->d_tconst + (size_t)2 * t_exp * c->Ltot,
                     c->d_prime);
}

void mod_down_final(bgv_ctx* c, const uint64_t* u, const uint64_t* dl, const uint64_t* add, int64_t add_stride,
                    uint64_t* out, int n, int level, int t_exp) {
  // add_stride < 0 encodes "only component 0 gets an addend" with |add_stride| the ct stride
  int comps = add_stride < 0 ? 1 : 2;
  int64_t stride = add_stride < 0 ? -add_stride : add_stride;
  const double* pinv = c->d_moddown + c->prm.K + (size_t)c->prm.K * c->prm.L;
  hipLaunchKernelGGL(k_mod_down_final, grid_for(c->N, n * 2 * level), dim3(block_for(c->N)), 0, c->stream, u, dl, add,
                     stride, comps, out, level, c->N, c->prm.K, pinv,
                     c->d_tconst + ((size_t)2 * t_exp + 1) * c->Ltot, c->d_prime);
}

void msw_w(bgv_ctx* c, const uint64_t* top, uint64_t* w, int n, int level, int t_exp) {
  const double tinv_top = c->h_tinv[(size_t)t_exp * c->Ltot + (level - 1)];
  hipLaunchKernelGGL(k_msw_w, grid_for(c->N, n * 2), dim3(block_for(c->N)), 0, c->stream, top, w, level, c->N,
                     tinv_top, c->d_prime);
}

void msw_corr(bgv_ctx* c, const uint64_t* tl, uint64_t* e, int n, int level, int to, int t_exp) {
  hipLaunchKernelGGL(k_msw_corr, grid_for(c->N, n * 2), dim3(block_for(c->N)), 0, c->stream, tl, e, level, to, c->N,
                     c->d_msw, c->prm.L, c->d_tconst + (size_t)2 * t_exp * c->Ltot,
                     c->d_tconst + ((size_t)2 * t_exp + 1) * c->Ltot, c->d_prime);
}

void lincomb(bgv_ctx* c, const uint64_t* const* xs, const int* rows, int nt, const double* sc, int sc_stride,
             int cst_row, uint64_t* out, int n, int level) {
  LinTerms t;
  for (int i = 0; i < 16; ++i) {
    t.x[i] = i < nt ? xs[i] : nullptr;
    t.row[i] = i < nt ? rows[i] : 0;
  }
  hipLaunchKernelGGL(k_lincomb, grid_for(c->N, n * 2 * level), dim3(block_for(c->N)), 0, c->stream, t, nt, sc,
                     sc_stride, cst_row, out, level, c->N, c->d_prime);
}

void lincomb_multi(bgv_ctx* c, const LinMulti& m, int nt, int no, const double* sc, int sc_stride,
                   const double* scs, int n, int level) {
  if (scs)
    hipLaunchKernelGGL(k_lincomb_multi<true>, grid_for(c->N, n * 2 * level), dim3(block_for(c->N)), 0, c->stream, m,
                       nt, no, sc, sc_stride, scs, level, c->N, c->d_prime);
  else
    hipLaunchKernelGGL(k_lincomb_multi<false>, grid_for(c->N, n * 2 * level), dim3(block_for(c->N)), 0, c->stream, m,
                       nt, no, sc, sc_stride, scs, level, c->N, c->d_prime);
}

void ms_corr(bgv_ctx* c, const uint64_t* up, int64_t up_stride, const uint64_t* utop, int64_t ut_stride,
             const uint64_t* dtop, int64_t dt_stride, uint64_t* e, int n, int level, int t_exp) {
  hipLaunchKernelGGL(k_ms_corr, grid_for(c->N, n * 2), dim3(block_for(c->N)), 0, c->stream, up, up_stride, utop,
                     ut_stride, dtop, dt_stride, e, level, c->N, c->prm.K, c->prm.L, c->d_moddown,
                     c->d_mdfold + (size_t)t_exp * c->prm.K * c->prm.L, c->d_tconst + (size_t)2 * t_exp * c->Ltot,
                     c->d_tconst + ((size_t)2 * t_exp + 1) * c->Ltot, c->d_prime);
}

void batch_sum(bgv_ctx* c, const uint64_t* x, uint64_t* out, int n, int level) {
  hipLaunchKernelGGL(k_batch_sum, grid_for(c->N, 2 * level), dim3(block_for(c->N)), 0, c->stream, x, out, n, level,
                     c->N, c->d_prime);
}

void automorph(bgv_ctx* c, const uint64_t* x, int64_t xs, uint64_t* y, int64_t ys, int n, int rows, int g) {
  const int logB = c->logN < 12 ? c->logN : 12;  // 32 KiB of LDS per block
  const int B = 1 << logB;
  hipLaunchKernelGGL(k_automorph, dim3(c->N >> logB, n * rows), dim3(B < 256 ? B : 256), (size_t)B * 8, c->stream, x,
                     xs, y, ys, rows, c->logN, logB, (uint32_t)g);
}

void from_signed(bgv_ctx* c, const int64_t* v, uint64_t* y, int n_polys, int rows, LimbMap lm) {
  hipLaunchKernelGGL(k_from_signed, grid_for(c->N, n_polys * rows), dim3(block_for(c->N)), 0, c->stream, v, y, rows,
                     c->N, lm, c->d_prime);
}

void mul_pointwise(bgv_ctx* c, const uint64_t* a, const uint64_t* b, uint64_t* out, int n_limbs, LimbMap lm,
                   int64_t) {
  hipLaunchKernelGGL(k_mul_pointwise, grid_for(c->N, n_limbs), dim3(block_for(c->N)), 0, c->stream, a, b, out, c->N, lm,
                     c->d_prime);
}

void phase(bgv_ctx* c, const uint64_t* ct, const uint64_t* S, uint64_t* v, int n, int level) {
  hipLaunchKernelGGL(k_phase, grid_for(c->N, n * level), dim3(block_for(c->N)), 0, c->stream, ct, S, v, level, c->N,
                     c->d_prime);
}

void enc_combine(bgv_ctx* c, const uint64_t* M, const uint64_t* C1, const uint64_t* S, uint64_t* ct, int n) {
  hipLaunchKernelGGL(k_enc_combine, grid_for(c->N, n * c->prm.L), dim3(block_for(c->N)), 0, c->stream, M, C1, S, ct,
                     c->prm.L, c->N, c->d_prime);
}

void key_combine(bgv_ctx* c, const uint64_t* A, const uint64_t* S, const uint64_t* E, const uint64_t* Sp,
                 uint64_t* key, int dnum) {
  // tmod for t = p^r and P mod q_m live in the t-constant table and the ModDown table area
  const double* tmod_full = c->d_tconst + ((size_t)2 * c->prm.r + 1) * c->Ltot;
  const double* pmod = c->d_moddown + c->prm.K + (size_t)c->prm.K * c->prm.L + c->prm.L;
  hipLaunchKernelGGL(k_key_combine, grid_for(c->N, dnum * c->Ltot), dim3(block_for(c->N)), 0, c->stream, A, S, E, Sp,
                     key, c->Ltot, c->prm.L, c->N, c->alpha, 0.0, tmod_full, pmod, c->d_prime);
}

}  // namespace lk

// ------------------------------------------------------------------ allocation-free scratch
namespace {
// Scratch of the allocation-free entry points: BGV_NOALLOC_SCRATCH_WORDS words on every GPU
// the library runs on, held by the loaded code object until the process ends and shared by
// every call on that GPU.  In host code this name is only a host-side stand-in: the device
// address comes from hipGetSymbolAddress, once per device, and only that address is used.
__device__ __align__(256) uint64_t scratch[BGV_NOALLOC_SCRATCH_WORDS];
std::mutex g_scratch_mu;
constexpr int MAX_DEVICES = 64;
uint64_t* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

uint64_t* noalloc_scratch_ptr(int* device) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  if (device) *device = dev;
  std::lock_guard<std::mutex> guard(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = (uint64_t*)p;
  }
  return g_scratch_ptr[dev];
}
