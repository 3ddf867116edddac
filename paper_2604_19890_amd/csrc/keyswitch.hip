// Key-switching kernels built on the transform's passes (gfx950): the ModUp fused with the
// passes around it, and the second forward pass fused with the key inner product.
#include "ctx.hpp"
#include "ntt_layout.hpp"
#include "ntt_stages.hpp"

namespace {

using namespace nttl;

// Second forward pass fused with the key-switching inner product, over the
// ModUp output y [n][dn][rows][N] whose first pass is done.  The rows of a
// digit's own primes are not in y: they are the input x itself (evaluation form,
// [n][level][N] at ciphertext stride xs) and are used as they are.  A block
// handles one (row block, target row m, ciphertext): for every digit j it
// finishes the transform of y[ct][j][m] in registers and LDS, multiplies it by
// key[j][comp][prime(m)] and accumulates; u[ct][comp][m] receives the sums.
// Block order: workgroups are dispatched round-robin over the eight XCDs, so the
// blocks of one (row block, m) group -- which read the same key rows -- are given
// ids with the same residue mod 8 and consecutive positions on that XCD; the key
// rows are then read once into that XCD's L2 and shared by all ciphertexts.
template <int LOGS>
__global__ void __launch_bounds__(NT_MAX) k_ntt2_key_inner(const uint64_t* __restrict__ y,
                                                           const uint64_t* __restrict__ xown, int64_t xs,
                                                           const uint64_t* __restrict__ key,
                                                           uint64_t* __restrict__ u, int logN, int s0, int level,
                                                           int dn, int K, int alpha, int Lfull, int Ltot, int n_ct,
                                                           const PrimeD* __restrict__ pc,
                                                           const double* __restrict__ tw,
                                                           const uint64_t* __restrict__ dtop, int64_t dtop_ct,
                                                           int64_t dtop_comp, double pmod_top, int inv_from,
                                                           const double* __restrict__ itw) {
  constexpr int S = 1 << LOGS;
  constexpr int T = S / 16;
  constexpr int T_LOG = LOGS - 4;
  __shared__ double lds[NT_MAX * 16 + NT_MAX + NT_MAX];
  const int N = 1 << logN;
  const int NT = blockDim.x;
  const int SUBS = NT / T;
  const int rows = level + K;
  const int RB = (N / S) / SUBS;  // row blocks per limb
  const int G = RB * rows;         // (row block, m) groups
  const int wid = blockIdx.x;
  int g, ct;
  if ((G & 7) == 0) {
    const int k = wid >> 3;
    g = (wid & 7) + 8 * (k / n_ct);
    ct = k % n_ct;
  } else {
    g = wid / n_ct;
    ct = wid % n_ct;
  }
  const int rb = g % RB;
  const int m = g / RB;
  const int pm = m < level ? m : Lfull + (m - level);
  const double q = pc[pm].q, qinv = pc[pm].qinv;
  const double* __restrict__ w = tw + (size_t)pm * N;
  const int tmax_log = logN - s0 - 1;  // tmin = 1 in the second pass
  const int tau = threadIdx.x % T;
  const int sl = threadIdx.x / T;
  const int st = rb * SUBS + sl;
  const int base = st << (tmax_log + 1);
  const int g1 = base + tau;
  const int gs1_log = T_LOG;
  const int g2 = base + 16 * tau;
  double acc0[16], acc1[16], v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc0[i] = acc1[i] = 0.0;
  // the first four stages' twiddles depend on the sub-transform only, the same for every digit:
  // loaded once, so a digit's transform starts without waiting for memory
  double tw1[15];
  ct_twiddles<8>(tw1, w, N, g1, gs1_log);
  // Digit j + 1's y row is requested at the start of digit j, in the same batch
  // as digit j's last-four-stage twiddle loads (the first four stages' twiddles are
  // held in registers): loads complete in issue order, so the transform waits for
  // both, and each digit costs one round trip to memory for its data and twiddles
  // instead of two.
  const uint64_t* __restrict__ yrow = y + ((size_t)ct * dn * rows + m) * N + g1;
  const size_t ystep = (size_t)rows * N;
  const int own_j = m < level ? m / alpha : -1;  // the digit whose own prime m is
  const uint64_t* __restrict__ xrow = xown + (size_t)ct * xs + (size_t)m * N + g1;
  uint64_t yn[16];
  {
    const uint64_t* __restrict__ yp = own_j == 0 ? xrow : yrow;
#pragma unroll
    for (int i = 0; i < 16; ++i) yn[i] = __builtin_nontemporal_load(&yp[(size_t)i << gs1_log]);
  }
  for (int j = 0; j < dn; ++j) {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = u2d(yn[i]);
    if (j + 1 < dn) {
      const uint64_t* __restrict__ yp = own_j == j + 1 ? xrow : yrow + (size_t)(j + 1) * ystep;
#pragma unroll
      for (int i = 0; i < 16; ++i) yn[i] = __builtin_nontemporal_load(&yp[(size_t)i << gs1_log]);
    }
    if (j != own_j) {
      ct_stages_tw<8>(v, tw1, q, qinv);
      if (T > 1) {  // with T = 1 the four register stages were all of the pass
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = red(v[i], q, qinv);
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
        ct_stages<(T > 1 ? T / 2 : 1)>(v, w, N, g2, 0, q, qinv);
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
        wave_lds_sync();  // the next digit writes the same LDS rows
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = red(v[i], q, qinv);
    }
    const uint64_t* __restrict__ kb = key + (((size_t)j * 2 + 0) * Ltot + pm) * N + g1;
    const uint64_t* __restrict__ ka = key + (((size_t)j * 2 + 1) * Ltot + pm) * N + g1;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      acc0[i] += mul_lazy(v[i], u2d(kb[(size_t)i << gs1_log]), q, qinv);
      acc1[i] += mul_lazy(v[i], u2d(ka[(size_t)i << gs1_log]), q, qinv);
    }
    if ((j & 3) == 3) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        acc0[i] = red(acc0[i], q, qinv);
        acc1[i] = red(acc1[i], q, qinv);
      }
    }
  }
  // The product step's switch drops the top prime: there u's top row leaves as
  // u_top + P d_top (d_top: the tensor's top row, evaluation form), which carries d_top
  // through the inverse transform of u's top row instead of a transform of its own.
  if (dtop && m == level - 1) {
    const uint64_t* __restrict__ d0 = dtop + (size_t)ct * dtop_ct + g1;
    const uint64_t* __restrict__ d1 = d0 + dtop_comp;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      acc0[i] += mul_lazy(u2d(d0[(size_t)i << gs1_log]), pmod_top, q, qinv);
      acc1[i] += mul_lazy(u2d(d1[(size_t)i << gs1_log]), pmod_top, q, qinv);
    }
  }
  uint64_t* __restrict__ u0 = u + ((size_t)ct * 2 * rows + m) * N + g1;
  uint64_t* __restrict__ u1 = u0 + (size_t)rows * N;
  if (inv_from >= 0 && m >= inv_from) {
    // Rows that go on to coefficient form: the first pass of their inverse transform (the
    // contiguous pass, the geometry of this one) is run here on the canonical sums, as the
    // separate pass would run it on the stored words.
    const double* __restrict__ iw = itw + (size_t)pm * N;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      double* acc = comp == 0 ? acc0 : acc1;
      uint64_t* __restrict__ up = comp == 0 ? u0 : u1;
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = canon(red(acc[i], q, qinv), q);
      if (T > 1) {  // with T = 1 the four register stages are the whole pass
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = v[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
        gs_stages<(T > 1 ? T / 2 : 1)>(v, iw, N, g2, 0, q, qinv);
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
      }
      gs_stages<8>(v, iw, N, g1, gs1_log, q, qinv);
#pragma unroll
      for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(d2u(canon(red(v[i], q, qinv), q)), &up[(size_t)i << gs1_log]);
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    u0[(size_t)i << gs1_log] = to_u(acc0[i], q, qinv);
    u1[(size_t)i << gs1_log] = to_u(acc1[i], q, qinv);
  }
}

// ModUp fused with the transform passes around it.  The key switch of x (evaluation form,
// [n][level][N]) needs x in coefficient form, the ModUp of each digit to the other primes, and
// the forward transform of every ModUp row.  After the first (contiguous) pass of x's inverse
// transform, written to xh, a block takes one column block of one digit j of one ciphertext:
//  * it finishes the inverse transform of the digit's source rows there (the column pass) and
//    scales them by N^-1 Qhat_i^-1 (one folded constant per row), which gives the ModUp
//    operands v_i = [x_i Qhat_i^-1]_{q_i} in [0, q_i); they stay in registers;
//  * for every target row m outside the digit it forms sum_i v_i (Qhat_i mod q_m) and runs the
//    first (column) pass of the forward transform under q_m on it, and writes y[ct][j][m].
// y then holds what the separate ModUp and first forward pass would have written (canonical
// residues of the same exact values), while x's coefficient form and the untransformed ModUp
// rows are never stored.  The second pass, fused with the key inner product, follows.
// With ALPHA = 6 the operands of the last source row are kept in LDS (each thread reads back
// only its own words, so no barrier is needed for them): the other five rows and the working
// registers then fit two waves per SIMD.  blockIdx.z splits the target rows into gridDim.z
// contiguous ranges (each block redoes the digit's source rows): small batches then still
// fill the chip.
template <int LOGS, int ALPHA>
__global__ void __launch_bounds__(NT_MAX, 2) k_modup_cols(const uint64_t* __restrict__ xh, uint64_t* __restrict__ y,
                                                       int logN, int level, int dn, int dnum, int alpha, int K,
                                                       int Lfull, int Ltot, const double* __restrict__ mu_scale,
                                                       const double* __restrict__ modup,
                                                       const PrimeD* __restrict__ pc, const double* __restrict__ tw,
                                                       const double* __restrict__ itw) {
  constexpr int S = 1 << LOGS;
  constexpr int T = S / 16;
  constexpr int T_LOG = LOGS - 4;
  __shared__ double lds[NT_MAX * 16 + NT_MAX + NT_MAX];
  const int N = 1 << logN;
  const int NT = blockDim.x;
  const int SUBS = NT / T;
  const int ct = blockIdx.y / dn;
  const int j = blockIdx.y % dn;
  const int lo = j * alpha;
  const int na = min(lo + alpha, level) - lo;
  const int rows = level + K;
  // column pass geometry (first forward / last inverse pass: stages 0 .. LOGS-1)
  const int tmax_log = logN - 1;
  const int tmin_log = logN - LOGS;
  const int sl = threadIdx.x % SUBS;
  const int tau = threadIdx.x / SUBS;
  const int bx = (blockIdx.x + blockIdx.y) & (gridDim.x - 1);
  const int st = bx * SUBS + sl;
  const int lo_c = st & ((1 << tmin_log) - 1);
  const int hi_c = st >> tmin_log;
  const int base = (hi_c << (tmax_log + 1)) + lo_c;
  const int g1 = base + (tau << tmin_log);
  const int gs1_log = T_LOG + tmin_log;
  const int g2 = base + ((16 * tau) << tmin_log);
  constexpr int LSRC = ALPHA == 6 ? 1 : 0;  // source rows held in LDS
  constexpr int RSRC = ALPHA - LSRC;          // source rows held in registers
  __shared__ double lsrc[LSRC > 0 ? LSRC * 16 * NT_MAX : 1];
  double src[RSRC][16];
  // tables of (level, digit): the folded scales [alpha] and ModUp's Qhat_i mod prime [alpha][Ltot]
  const size_t tab = (size_t)level * dnum + j;
  // Both passes read only the twiddles w[1 .. S) of their prime (S = 2^LOGS <= NT).  They are
  // staged in LDS, one row ahead: a thread loads one word of the next row's table at the top
  // of a row and stores it after the row's second barrier, when the readers of that buffer in
  // the row before are done; the row's third barrier publishes it.  The last source row
  // stages the first target's (forward) table.
  static_assert(T > 1, "the staged twiddles rely on the exchange barriers");
  __shared__ double ltw[2][S];
  const double* __restrict__ basis = modup + tab * (size_t)alpha * (1 + Ltot) + alpha;
  uint64_t* __restrict__ yb = y + ((size_t)ct * dn + j) * rows * N + g1;
  const int per = (rows + gridDim.z - 1) / gridDim.z;
  const int m_end = min(rows, ((int)blockIdx.z + 1) * per);
  auto skip_digit = [&](int m) { return (m >= lo && m < lo + na) ? lo + na : m; };
  auto prime_of = [&](int m) { return m < level ? m : Lfull + (m - level); };
  int m = skip_digit(blockIdx.z * per);
  const bool lane_stages = (int)threadIdx.x < S;
  if (lane_stages) ltw[0][threadIdx.x] = itw[(size_t)lo * N + threadIdx.x];
  __syncthreads();
  int buf = 0;
  // ---- the digit's source rows: last inverse pass, scaled to the ModUp operands
#pragma unroll
  for (int a = 0; a < ALPHA; ++a) {
    if (a < na) {
      const int pi = lo + a;
      const double q = pc[pi].q, qinv = pc[pi].qinv;
      const double* w = ltw[buf];
      const bool last = a + 1 == na;
      const bool stage = lane_stages && (!last || m < m_end);
      const double pre = !stage ? 0.0 : last ? tw[(size_t)prime_of(m) * N + threadIdx.x]
                                             : itw[(size_t)(pi + 1) * N + threadIdx.x];
      const uint64_t* xp = xh + ((size_t)ct * level + pi) * N + g1;
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = u2d(__builtin_nontemporal_load(&xp[(size_t)i << gs1_log]));
      __syncthreads();  // the previous pass's last LDS reads are done
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = v[i];
      __syncthreads();
      if (stage) ltw[buf ^ 1][threadIdx.x] = pre;
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
      gs_stages<T / 2>(v, w, N, g2, tmin_log, q, qinv);
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
      gs_stages<8>(v, w, N, g1, gs1_log, q, qinv);
      buf ^= 1;
      const double sc = mu_scale[tab * alpha + a];  // N^-1 Qhat_i^-1 mod q_i
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const double o = canon(red(mul_lazy(red(v[i], q, qinv), sc, q, qinv), q, qinv), q);
        if (a < RSRC) src[a < RSRC ? a : 0][i] = o;
        else lsrc[((a - RSRC) * 16 + i) * NT_MAX + threadIdx.x] = o;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (a < RSRC) src[a < RSRC ? a : 0][i] = 0.0;
        else lsrc[((a - RSRC) * 16 + i) * NT_MAX + threadIdx.x] = 0.0;
      }
    }
  }
  // ---- every target row outside the digit: ModUp value, first forward pass, store
  for (; m < m_end; buf ^= 1) {
    const int mn = skip_digit(m + 1);
    const bool stage = mn < m_end && (int)threadIdx.x < S;
    const double pre = stage ? tw[(size_t)prime_of(mn) * N + threadIdx.x] : 0.0;
    const int pm = prime_of(m);
    const double q = pc[pm].q, qinv = pc[pm].qinv;
    const double* w = ltw[buf];
    // Branch-free over the digit's ALPHA slots: in a shorter last digit (na < ALPHA) the
    // missing sources are zero and so are their rows of the table (it is zero-filled), so
    // their terms add exact zeros; every slot's products can then be interleaved.
    double bm[ALPHA];
#pragma unroll
    for (int a = 0; a < ALPHA; ++a) bm[a] = basis[(size_t)a * Ltot + pm];
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < ALPHA; ++a) {
        const double x = a < RSRC ? src[a < RSRC ? a : 0][i] : lsrc[((a - RSRC) * 16 + i) * NT_MAX + threadIdx.x];
        acc += mul_lazy(x, bm[a], q, qinv);
      }
      v[i] = red(acc, q, qinv);
    }
    ct_stages<8>(v, w, N, g1, gs1_log, q, qinv);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = red(v[i], q, qinv);
    __syncthreads();
    if (stage) ltw[buf ^ 1][threadIdx.x] = pre;
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
    ct_stages<T / 2>(v, w, N, g2, tmin_log, q, qinv);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
    uint64_t* yp = yb + (size_t)m * N;
#pragma unroll
    for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(d2u(canon(red(v[i], q, qinv), q)), &yp[(size_t)i << gs1_log]);
    m = mn;
  }
}

// ModDown merged with the switch, fused with the transform passes around it (the mirror of
// k_modup_cols).  u [n][2][rows][N] holds u's top row (u_top + P d_top) and K special rows after
// the first pass of their inverse transform.  A block takes one column block of one polynomial
// cc = ct * 2 + comp:
//  * the last inverse pass of the K special rows, each scaled to v_k = [u_k t^-1 Phat_k^-1]_{p_k}
//    (N^-1 folded into the same constant), and of the top row, which gives the switch's centered
//    w from u_top + P d_top and the ModDown conversion of the v_k at the top prime;
//  * for every target row i < level - 1: e_i = sum_k v_k [Phat_k t P^-1]_{q_i} + t w, the first
//    forward pass of e_i under q_i, and the store.
// e [n][2][level-1][N] then holds what the merged correction and the first forward pass would
// have written.  Three of the K converted rows and w's row stay in registers, the others in
// LDS (96 KiB at K = 6); one block per CU.
template <int LOGS, int KK>
__global__ void __launch_bounds__(NT_MAX, 1) k_moddown_cols(const uint64_t* __restrict__ u, uint64_t* __restrict__ e,
                                                         int logN, int level, int rows, int Lfull,
                                                         const double* __restrict__ md,
                                                         const double* __restrict__ mdfold,
                                                         const double* __restrict__ tinv,
                                                         const double* __restrict__ tmod,
                                                         const PrimeD* __restrict__ pc, const double* __restrict__ tw,
                                                         const double* __restrict__ itw) {
  constexpr int S = 1 << LOGS;
  constexpr int T = S / 16;
  constexpr int T_LOG = LOGS - 4;
  static_assert(T > 1, "the staged twiddles rely on the exchange barriers");
  __shared__ double lds[NT_MAX * 16 + NT_MAX + NT_MAX];
  __shared__ double ltw[2][S];
  const int N = 1 << logN;
  const int NT = blockDim.x;
  const int SUBS = NT / T;
  const int cc = blockIdx.y;
  const int tmax_log = logN - 1;
  const int tmin_log = logN - LOGS;
  const int sl = threadIdx.x % SUBS;
  const int tau = threadIdx.x / SUBS;
  const int bx = (blockIdx.x + blockIdx.y) & (gridDim.x - 1);
  const int st = bx * SUBS + sl;
  const int lo_c = st & ((1 << tmin_log) - 1);
  const int hi_c = st >> tmin_log;
  const int base = (hi_c << (tmax_log + 1)) + lo_c;
  const int g1 = base + (tau << tmin_log);
  const int gs1_log = T_LOG + tmin_log;
  const int g2 = base + ((16 * tau) << tmin_log);
  const double* phat_inv = md;
  const double* phat_mod = md + KK;
  const double* pinv = md + KK + (size_t)KK * Lfull;
  const uint64_t* __restrict__ ub = u + (size_t)cc * rows * N + g1;
  // the last inverse (column) pass of one row in place on v, as the separate pass runs it
  auto inverse_last_pass = [&](double* v, const double* __restrict__ w, double q, double qinv) {
    __syncthreads();  // the previous row's last LDS reads are done
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
    gs_stages<T / 2>(v, w, N, g2, tmin_log, q, qinv);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
    gs_stages<8>(v, w, N, g1, gs1_log, q, qinv);
  };
  constexpr int RS = KK < 3 ? KK : 3;  // converted rows held in registers; the rest in LDS
  __shared__ double lsrc[(KK > RS ? KK - RS : 1) * 16 * NT_MAX];
  double vk[RS][16];
  auto src = [&](int k, int i) -> double {
    return k < RS ? vk[k < RS ? k : 0][i] : lsrc[((k - RS) * 16 + i) * NT_MAX + threadIdx.x];
  };
#pragma unroll
  for (int k = 0; k < KK; ++k) {
    const int pk = Lfull + k;
    const double q = pc[pk].q, qinv = pc[pk].qinv;
    // N^-1 t^-1 Phat_k^-1 mod p_k
    const double sc = canon(red(mul_lazy(canon(red(mul_lazy(pc[pk].ninv, tinv[pk], q, qinv), q, qinv), q),
                                         phat_inv[k], q, qinv), q, qinv), q);
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = u2d(__builtin_nontemporal_load(&ub[(size_t)(level + k) * N + ((size_t)i << gs1_log)]));
    inverse_last_pass(v, itw + (size_t)pk * N, q, qinv);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double o = canon(red(mul_lazy(red(v[i], q, qinv), sc, q, qinv), q, qinv), q);
      if (k < RS) vk[k < RS ? k : 0][i] = o;
      else lsrc[((k - RS) * 16 + i) * NT_MAX + threadIdx.x] = o;
    }
  }
  double wms[16];
  {
    const int it = level - 1;
    const double q = pc[it].q, qinv = pc[it].qinv;
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = u2d(__builtin_nontemporal_load(&ub[(size_t)it * N + ((size_t)i << gs1_log)]));
    inverse_last_pass(v, itw + (size_t)it * N, q, qinv);
    const double ninv = pc[it].ninv, tm = tmod[it], pv = pinv[it], ti = tinv[it];
    double pm[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) pm[k] = phat_mod[(size_t)k * Lfull + it];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double ut = red(mul_lazy(red(v[i], q, qinv), ninv, q, qinv), q, qinv);  // u_top + P d_top
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < KK; ++k) acc += mul_lazy(src(k, i), pm[k], q, qinv);
      const double wt = canon(red(acc, q, qinv), q);
      const double diff = red(ut - mul_lazy(wt, tm, q, qinv), q, qinv);
      const double o = canon(red(mul_lazy(diff, pv, q, qinv), q, qinv), q);
      const double w = canon(mul_lazy(o, ti, q, qinv), q);
      wms[i] = w > (q - 1.0) * 0.5 ? w - q : w;  // centered
    }
  }
  // ---- targets: the correction of every row below the top, its first forward pass, store
  const int nt = level - 1;
  const int per = (nt + gridDim.z - 1) / gridDim.z;
  const int i_end = min(nt, ((int)blockIdx.z + 1) * per);
  int i = blockIdx.z * per;
  const bool lane_stages = (int)threadIdx.x < S;
  if (i < i_end && lane_stages) ltw[0][threadIdx.x] = tw[(size_t)i * N + threadIdx.x];
  __syncthreads();
  for (int buf = 0; i < i_end; ++i, buf ^= 1) {
    const bool stage = i + 1 < i_end && lane_stages;
    const double pre = stage ? tw[(size_t)(i + 1) * N + threadIdx.x] : 0.0;
    const double q = pc[i].q, qinv = pc[i].qinv;
    double f[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) f[k] = mdfold[(size_t)k * Lfull + i];
    const double tm = tmod[i];
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < KK; ++k) a += mul_lazy(src(k, j), f[k], q, qinv);
      const double b = mul_lazy(wms[j] < 0.0 ? wms[j] + q : wms[j], tm, q, qinv);
      v[j] = canon(red(red(a, q, qinv) + b, q, qinv), q);
    }
    const double* w = ltw[buf];
    ct_stages<8>(v, w, N, g1, gs1_log, q, qinv);
    // Every thread has left the previous row, the last reader of the other twiddle buffer: the
    // next row's table goes there now, and the barrier after the exchange writes publishes it.
    __syncthreads();
    if (stage) ltw[buf ^ 1][threadIdx.x] = pre;
#pragma unroll
    for (int j = 0; j < 16; ++j) lds[lds_idx(sl, tau + T * j, S)] = red(v[j], q, qinv);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds[lds_idx(sl, 16 * tau + j, S)];
    ct_stages<T / 2>(v, w, N, g2, tmin_log, q, qinv);
    // stored from the second layout (16 adjacent columns per store, as from the first): without
    // the exchange back, a row costs one barrier and 32 LDS accesses less
    uint64_t* ep = e + (size_t)cc * nt * N + g2 + (size_t)i * N;
#pragma unroll
    for (int j = 0; j < 16; ++j) __builtin_nontemporal_store(d2u(canon(red(v[j], q, qinv), q)), &ep[(size_t)j << tmin_log]);
  }
}

}  // namespace

namespace lk {

bool ntt_fused_inner_ok(const bgv_ctx* c) { return c->logN > 8; }

bool modup_cols_ok(const bgv_ctx* c) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  const int A = c->alpha;
  return c->modup_fused && p2 > 0 && p1 >= 5 && p1 <= 8 && (A == 1 || A == 2 || A == 4 || A == 6) &&
         c->d_modup_scale != nullptr;
}

void modup_cols(bgv_ctx* c, const uint64_t* xh, uint64_t* y, int n, int level) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  const int N = c->N, A = c->alpha, K = c->prm.K;
  const int dn = (level + A - 1) / A;
  const int S = 1 << p1, T = S / 16;
  const int NT = N / 16 < NT_MAX ? N / 16 : NT_MAX;
  const int SUBS = NT / T;
  // the target rows of each (ciphertext, digit) over up to 4 blocks while the grid is under
  // 1024 blocks (four per compute unit)
  const int base_blocks = ((N / S) / SUBS) * n * dn;
  int split = 1;
  while (split < 4 && base_blocks * split < 1024) split *= 2;
  dim3 grid((N / S) / SUBS, n * dn, split);
#define MU_CASE(LS, AL)                                                                                        \
  if (p1 == LS && A == AL) {                                                                                   \
    hipLaunchKernelGGL((k_modup_cols<LS, AL>), grid, dim3(NT), 0, c->stream, xh, y, c->logN, level, dn, c->dnum, \
                       A, K, c->prm.L, c->Ltot, c->d_modup_scale, c->d_modup, c->d_prime, c->d_tw, c->d_itw);   \
    return;                                                                                                    \
  }
#define MU_ALPHAS(LS) MU_CASE(LS, 1) MU_CASE(LS, 2) MU_CASE(LS, 4) MU_CASE(LS, 6)
  MU_ALPHAS(5)
  MU_ALPHAS(6)
  MU_ALPHAS(7)
  MU_ALPHAS(8)
#undef MU_ALPHAS
#undef MU_CASE
}

bool moddown_cols_ok(const bgv_ctx* c, int n) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  if (c->moddown_fused == 0 || p2 <= 0 || p1 < 5 || p1 > 8 || c->prm.K < 1 || c->prm.K > 6) return false;
  if (c->moddown_fused == 2) return true;
  // one block per CU runs (one wave per SIMD): on a smaller grid the separate launches are faster
  // (measured at N = 2^16: the fused product step slower by 1-25% up to 8 ciphertexts, even at 16)
  const int S = 1 << p1, T = S / 16;
  const int NT = c->N / 16 < NT_MAX ? c->N / 16 : NT_MAX;
  return (int64_t)((c->N / S) / (NT / T)) * n * 2 >= 512;
}

void moddown_cols(bgv_ctx* c, const uint64_t* u, uint64_t* e, int n, int level, int t_exp) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  const int N = c->N, K = c->prm.K, L = c->prm.L, rows = level + K;
  const int S = 1 << p1, T = S / 16;
  const int NT = N / 16 < NT_MAX ? N / 16 : NT_MAX;
  const int SUBS = NT / T;
  // one block per CU: spread the target rows over up to 8 blocks while the grid is small
  const int base_blocks = ((N / S) / SUBS) * n * 2;
  int split = 1;
  while (split < 8 && base_blocks * split < 512 && (level - 1) / (split * 2) >= 1) split *= 2;
  dim3 grid((N / S) / SUBS, n * 2, split);
  const double* mdfold = c->d_mdfold + (size_t)t_exp * K * L;
  const double* tinv = c->d_tconst + (size_t)2 * t_exp * c->Ltot;
  const double* tmod = c->d_tconst + ((size_t)2 * t_exp + 1) * c->Ltot;
#define MD_CASE(LS, KKK)                                                                                           \
  if (p1 == LS && K == KKK) {                                                                                      \
    hipLaunchKernelGGL((k_moddown_cols<LS, KKK>), grid, dim3(NT), 0, c->stream, u, e, c->logN, level, rows, L,       \
                       c->d_moddown, mdfold, tinv, tmod, c->d_prime, c->d_tw, c->d_itw);                           \
    return;                                                                                                        \
  }
#define MD_KS(LS) MD_CASE(LS, 1) MD_CASE(LS, 2) MD_CASE(LS, 3) MD_CASE(LS, 4) MD_CASE(LS, 5) MD_CASE(LS, 6)
  MD_KS(5)
  MD_KS(6)
  MD_KS(7)
  MD_KS(8)
#undef MD_KS
#undef MD_CASE
}

void ntt_pass1_key_inner(bgv_ctx* c, uint64_t* y, const uint64_t* x, int64_t x_ct_stride, const uint64_t* key,
                         uint64_t* u, int n, int level, bool pass1_done, const uint64_t* dtop, int64_t dtop_ct,
                         int64_t dtop_comp, double pmod_top, int inv_from) {
  const int logN = c->logN;
  int p1, p2;
  ntt_split(c, &p1, &p2);
  const int A = c->alpha, K = c->prm.K, L = c->prm.L;
  const int dn = (level + A - 1) / A, rows = level + K;
  // first pass over the non-own rows (unless the fused ModUp has done it)
  if (!pass1_done) ntt_forward_first_pass(c, y, n * dn * rows, LimbMap{rows, level, L, A, dn, 0, 0});
  const int N = c->N, S = 1 << p2, T = S / 16;
  const int NT = N / 16 < NT_MAX ? N / 16 : NT_MAX;
  const int SUBS = NT / T;
  dim3 grid(((N / S) / SUBS) * n * rows);
  switch (p2) {
#define CASE2(LS)                                                                                              \
  case LS:                                                                                                     \
    hipLaunchKernelGGL((k_ntt2_key_inner<LS>), grid, dim3(NT), 0, c->stream, y, x, x_ct_stride, key, u, logN, p1, \
                       level, dn, K, A, L, c->Ltot, n, c->d_prime, c->d_tw, dtop, dtop_ct, dtop_comp, pmod_top,     \
                       inv_from, c->d_itw);                                                                     \
    break;
    CASE2(4)
    CASE2(5)
    CASE2(6)
    CASE2(7)
    CASE2(8)
#undef CASE2
    default:
      break;
  }
}

}  // namespace lk
