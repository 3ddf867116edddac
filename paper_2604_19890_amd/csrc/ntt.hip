// Batched negacyclic NTT / INTT for gfx950.
//
// Forward transform (coefficients -> evaluation form, bit-reversed order):
// Cooley-Tukey butterflies (x, y) -> (x + w y, x - w y) over stages with
// half-distance t = N/2, N/4, .., 1; the butterfly whose upper element sits at
// index j uses w = psi^brv((N + j) / 2t).  Inverse: Gentleman-Sande butterflies
// (x, y) -> (x + y, (x - y) w^-1) over t = 1, .., N/2 with the table of psi^-brv,
// then a factor N^-1.  The result is the evaluation of the polynomial at
// psi^(2 brv(j) + 1) in slot j.
//
// Work split: the log2 N stages are done in one pass (N <= 256) or two passes
// of S = 2^LOGS points each (first pass: "columns" of stride N/S, second pass:
// contiguous blocks).  In a pass every sub-transform of S points belongs to
// S/16 threads holding 16 values each in registers: four stages run in
// registers on values S/16 apart, one LDS exchange regroups each thread onto 16
// consecutive points for the remaining stages, and a second exchange restores
// the coalesced order for the store.  Global loads and stores are coalesced:
// in the column pass neighbouring threads handle neighbouring columns, in the
// contiguous pass neighbouring threads handle neighbouring points.
//
// Reduction is lazy.  A Cooley-Tukey step of four register stages starts with
// |v| <= q and keeps every value below 7.1 q without reducing: at the four
// stages the multiplicand is below 1, 1.9, 3.1 and 4.8 q; the quotient estimate
// of a product is off by at most 3 * 2^-53 |y w / q| + 1/2, so the product's
// representative stays below 0.9, 1.2, 1.7 and 2.3 q, and every intermediate
// (including |h - k q| <= 2.3 q + ulp(h)/2 < 2^53) is exact.  A Gentleman-Sande
// step reduces the sums after its second and fourth stage, which keeps every
// value below 4 q and every multiplicand below 8 q.  Each step ends with one
// reduction of its 16 values.
#include "ctx.hpp"
#include "ntt_stages.hpp"

namespace {

constexpr int NT_MAX = 256;

__device__ __forceinline__ int lds_idx(int sl, int k, int S) { return sl * (S + (S >> 4) + 1) + k + (k >> 4); }

// Ordering point for an LDS exchange among the lanes of one wavefront.  The LDS
// instructions of a wave are performed in issue order, so it suffices to keep
// the compiler from moving LDS accesses across this point; no s_barrier is
// issued and the other waves of the block run on.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS exchange point of a pass.  In a contiguous pass (tmin = 1) the T <= 16
// threads of a sub-transform are consecutive lanes of one wave (T divides 64)
// and each sub-transform has LDS rows of its own, so the exchange stays inside
// the wave; a column pass spreads a sub-transform over the block's waves.
__device__ __forceinline__ void pass_sync(bool wave_local) {
  if (wave_local)
    wave_lds_sync();
  else
    __syncthreads();
}

// One pass over one block of one limb.  The pass reads from src (data itself when src
// is null, the transform then being in place) and writes to data, or with EPI (the last
// forward pass) applies the epilogue ep and writes ep.out.  `limb` is the launch limb
// index (after the block-row order below) and `bx` the block's position within the limb.
template <int LOGS, bool INV, bool EPI>
__device__ __forceinline__ void ntt_pass_body(uint64_t* data, const uint64_t* src, int logN, int s0,
                                              const LimbMap& lm, const PrimeD* __restrict__ pc,
                                              const double* __restrict__ tw, int last, const lk::NttEpi& ep,
                                              int limb, int bx, double* lds) {
  constexpr int S = 1 << LOGS;
  constexpr int T = S / 16;
  constexpr int T_LOG = LOGS - 4;
  const int N = 1 << logN;
  const int NT = blockDim.x;
  const int SUBS = NT / T;
  const int pi = limb_prime(lm, limb);
  const double q = pc[pi].q, qinv = pc[pi].qinv;
  const double* __restrict__ w = tw + (size_t)pi * N;
  const size_t row = (size_t)limb_phys(lm, limb) * N;
  uint64_t* x = data + row;
  const uint64_t* xs = src ? src + (size_t)limb_src(lm, limb) * N : data + row;
  const int tmax_log = logN - s0 - 1;
  const int tmin_log = logN - s0 - LOGS;
  const int tmin = 1 << tmin_log;
  int sl, tau;
  if (tmin == 1) {
    tau = threadIdx.x % T;
    sl = threadIdx.x / T;
  } else {
    sl = threadIdx.x % SUBS;
    tau = threadIdx.x / SUBS;
  }
  const int st = bx * SUBS + sl;
  const int lo = st & (tmin - 1);
  const int hi = st >> tmin_log;
  const int base = (hi << (tmax_log + 1)) + lo;
  // coalesced layout: register i holds global index g1 + i * 2^gs1_log
  const int g1 = base + (tau << tmin_log);
  const int gs1_log = T_LOG + tmin_log;
  // consecutive layout: register i holds global index g2 + i * tmin
  const int g2 = base + ((16 * tau) << tmin_log);
  uint64_t* xp = x + g1;
  const uint64_t* xsp = xs + g1;
  const bool wave_local = tmin == 1;
  double v[16];

#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = u2d(__builtin_nontemporal_load(&xsp[(size_t)i << gs1_log]));
  // the epilogue's rows are requested with the pass's own, so that they arrive
  // while the butterflies run
  uint64_t av[EPI ? 16 : 1], bv[EPI ? 16 : 1];
  int ii = 0;
  if constexpr (EPI) {
    const int gl = limb + lm.offset;
    const int cc = gl / ep.rows;
    ii = gl - cc * ep.rows;
    const size_t rr = (size_t)ii * N + g1;
    const uint64_t* ap = ep.a + (size_t)cc * ep.a_cc + rr;
#pragma unroll
    for (int i = 0; i < 16; ++i) av[i] = __builtin_nontemporal_load(&ap[(size_t)i << gs1_log]);
    if (ep.b) {
      const uint64_t* bp = ep.b + (size_t)cc * ep.b_cc + rr;
#pragma unroll
      for (int i = 0; i < 16; ++i) bv[i] = __builtin_nontemporal_load(&bp[(size_t)i << gs1_log]);
    }
  }

  if (!INV) {
    ct_stages<8>(v, w, N, g1, gs1_log, q, qinv);
    if (T > 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = red(v[i], q, qinv);
      pass_sync(wave_local);
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
      ct_stages<(T > 1 ? T / 2 : 1)>(v, w, N, g2, tmin_log, q, qinv);
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
      pass_sync(wave_local);
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
    }
  } else {
    if (T > 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = v[i];
      pass_sync(wave_local);
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
      gs_stages<(T > 1 ? T / 2 : 1)>(v, w, N, g2, tmin_log, q, qinv);
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
      pass_sync(wave_local);
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
    }
    gs_stages<8>(v, w, N, g1, gs1_log, q, qinv);
    if (last) {
      const double ninv = pc[pi].ninv;
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = mul_lazy(red(v[i], q, qinv), ninv, q, qinv);
    }
  }
  if constexpr (EPI) {
    uint64_t* op = ep.out + row + g1;
    const double qt = ep.qt[ii];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double e = canon(red(v[i], q, qinv), q);
      double s = u2d(av[i]) - (ep.sv ? mul_lazy(e, ep.sv[ii], q, qinv) : e);
      if (ep.b) s += mul_lazy(u2d(bv[i]), ep.sb[ii], q, qinv);
      __builtin_nontemporal_store(to_u(mul_lazy(red(s, q, qinv), qt, q, qinv), q, qinv), &op[(size_t)i << gs1_log]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(d2u(canon(red(v[i], q, qinv), q)), &xp[(size_t)i << gs1_log]);
  }
}

// Prime-major block order: consecutive block rows take the same limb position of
// consecutive polynomials, so the prime's twiddle table is read once into each XCD's L2
// and reused instead of cycling through every prime's table.
__device__ __forceinline__ int prime_major(const LimbMap& lm, int row, int rows) {
  if (rows % lm.period != 0) return row;
  const int polys = rows / lm.period;
  return (row % polys) * lm.period + row / polys;
}

// One pass over data as its own launch: block (x, y) takes block x of launch limb y.
template <int LOGS, bool INV, bool EPI>
__global__ void __launch_bounds__(NT_MAX) k_ntt_pass(uint64_t* data, const uint64_t* src, int logN, int s0,
                                                     LimbMap lm, const PrimeD* __restrict__ pc,
                                                     const double* __restrict__ tw, int last, lk::NttEpi ep) {
  __shared__ double lds[NT_MAX * 16 + NT_MAX + NT_MAX];
  const int limb = prime_major(lm, blockIdx.y, gridDim.y);
  if (limb_skipped(lm, limb)) return;
  // Column pass: the column block turns with the row.  Block ids go round-robin over the
  // eight XCDs, so with a fixed order an XCD would always take the same column blocks of
  // every row (16 blocks per row at N = 2^16); turning the order spreads them.
  const bool column = logN - s0 - LOGS > 0;
  const int bx = column ? ((blockIdx.x + blockIdx.y) & (gridDim.x - 1)) : blockIdx.x;
  ntt_pass_body<LOGS, INV, EPI>(data, src, logN, s0, lm, pc, tw, last, ep, limb, bx, lds);
}

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
                                                           const double* __restrict__ tw) {
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
  // Digit j + 1's y row is requested at the start of digit j, in the same batch
  // as digit j's twiddle loads: loads complete in issue order, so the transform
  // waits for both, and each digit costs one round trip to memory for its data
  // and twiddles instead of two.
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
      ct_stages<8>(v, w, N, g1, gs1_log, q, qinv);
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
  uint64_t* __restrict__ u0 = u + ((size_t)ct * 2 * rows + m) * N + g1;
  uint64_t* __restrict__ u1 = u0 + (size_t)rows * N;
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
// registers then fit two waves per SIMD.
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
  // ---- the digit's source rows: last inverse pass, scaled to the ModUp operands
#pragma unroll
  for (int a = 0; a < ALPHA; ++a) {
    if (a < na) {
      const int pi = lo + a;
      const double q = pc[pi].q, qinv = pc[pi].qinv;
      const double* __restrict__ w = itw + (size_t)pi * N;
      const uint64_t* xp = xh + ((size_t)ct * level + pi) * N + g1;
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = u2d(__builtin_nontemporal_load(&xp[(size_t)i << gs1_log]));
      if (T > 1) {
        __syncthreads();  // the previous pass's last LDS reads are done
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
        gs_stages<(T > 1 ? T / 2 : 1)>(v, w, N, g2, tmin_log, q, qinv);
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
      }
      gs_stages<8>(v, w, N, g1, gs1_log, q, qinv);
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
  const double* __restrict__ basis = modup + tab * (size_t)alpha * (1 + Ltot) + alpha;
  uint64_t* __restrict__ yb = y + ((size_t)ct * dn + j) * rows * N + g1;
  for (int m = 0; m < rows; ++m) {
    if (m >= lo && m < lo + na) continue;
    const int pm = m < level ? m : Lfull + (m - level);
    const double q = pc[pm].q, qinv = pc[pm].qinv;
    const double* __restrict__ w = tw + (size_t)pm * N;
    double bm[ALPHA];
#pragma unroll
    for (int a = 0; a < ALPHA; ++a) bm[a] = a < na ? basis[(size_t)a * Ltot + pm] : 0.0;
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < ALPHA; ++a) {
        if (a < na) {
          const double x = a < RSRC ? src[a < RSRC ? a : 0][i] : lsrc[((a - RSRC) * 16 + i) * NT_MAX + threadIdx.x];
          acc += mul_lazy(x, bm[a], q, qinv);
        }
      }
      v[i] = red(acc, q, qinv);
    }
    ct_stages<8>(v, w, N, g1, gs1_log, q, qinv);
    if (T > 1) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = red(v[i], q, qinv);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
      ct_stages<(T > 1 ? T / 2 : 1)>(v, w, N, g2, tmin_log, q, qinv);
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = red(v[i], q, qinv);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
    }
    uint64_t* yp = yb + (size_t)m * N;
#pragma unroll
    for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(d2u(canon(red(v[i], q, qinv), q)), &yp[(size_t)i << gs1_log]);
  }
}

template <bool INV>
void launch_pass(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm, int logS, int s0, int last,
                 const uint64_t* src = nullptr, const lk::NttEpi* epi = nullptr) {
  const int N = c->N;
  const int S = 1 << logS;
  const int T = S / 16;
  int NT = N / 16 < NT_MAX ? N / 16 : NT_MAX;
  const int SUBS = NT / T;
  dim3 grid((N / S) / SUBS, n_limbs);
  const double* tw = INV ? c->d_itw : c->d_tw;
  switch (logS) {
#define CASE(LS)                                                                                           \
  case LS:                                                                                                 \
    if constexpr (!INV) {                                                                                  \
      if (epi) {                                                                                           \
        hipLaunchKernelGGL((k_ntt_pass<LS, false, true>), grid, dim3(NT), 0, c->stream, d, src, c->logN, s0, \
                           lm, c->d_prime, tw, last, *epi);                                                \
        break;                                                                                             \
      }                                                                                                    \
    }                                                                                                      \
    hipLaunchKernelGGL((k_ntt_pass<LS, INV, false>), grid, dim3(NT), 0, c->stream, d, src, c->logN, s0, lm,  \
                       c->d_prime, tw, last, lk::NttEpi{});                                                \
    break;
    CASE(4)
    CASE(5)
    CASE(6)
    CASE(7)
    CASE(8)
#undef CASE
    default:
      break;
  }
}

}  // namespace

namespace lk {

void ntt_split(const bgv_ctx* c, int* p1, int* p2) {
  const int logN = c->logN;
  if (logN <= 8) {
    *p1 = logN;
    *p2 = 0;
    return;
  }
  int a = (logN + 1) / 2;
  if (c->ntt_split >= 4 && c->ntt_split <= 8 && logN - c->ntt_split >= 4 && logN - c->ntt_split <= 8) a = c->ntt_split;
  *p1 = a;
  *p2 = logN - a;
}

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
  dim3 grid((N / S) / SUBS, n * dn);
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

void ntt_inverse_first_pass(bgv_ctx* c, uint64_t* d, const uint64_t* src, int n_limbs, LimbMap lm) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  launch_pass<true>(c, d, n_limbs, lm, p2, p1, 0, src);
}

void ntt_pass1_key_inner(bgv_ctx* c, uint64_t* y, const uint64_t* x, int64_t x_ct_stride, const uint64_t* key,
                         uint64_t* u, int n, int level, bool pass1_done) {
  const int logN = c->logN;
  int p1, p2;
  ntt_split(c, &p1, &p2);
  const int A = c->alpha, K = c->prm.K, L = c->prm.L;
  const int dn = (level + A - 1) / A, rows = level + K;
  // first pass over the non-own rows (unless the fused ModUp has done it)
  if (!pass1_done) launch_pass<false>(c, y, n * dn * rows, LimbMap{rows, level, L, A, dn, 0, 0}, p1, 0, 0);
  const int N = c->N, S = 1 << p2, T = S / 16;
  const int NT = N / 16 < NT_MAX ? N / 16 : NT_MAX;
  const int SUBS = NT / T;
  dim3 grid(((N / S) / SUBS) * n * rows);
  switch (p2) {
#define CASE2(LS)                                                                                              \
  case LS:                                                                                                     \
    hipLaunchKernelGGL((k_ntt2_key_inner<LS>), grid, dim3(NT), 0, c->stream, y, x, x_ct_stride, key, u, logN, p1, \
                       level, dn, K, A, L, c->Ltot, n, c->d_prime, c->d_tw);                                   \
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

void ntt(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm, bool inverse, const uint64_t* src, const NttEpi* epi) {
  if (n_limbs <= 0) return;
  int p1, p2;
  ntt_split(c, &p1, &p2);
  // Two-pass transforms run chunk by chunk so that a chunk's first-pass output is
  // still in L2 / Infinity Cache when the second pass reads it.  The limb map is
  // shifted with the chunk: limb l of the chunk is limb off + l of the launch.
  // Transforms with a physical row placement, a separate source or an epilogue run whole.
  const bool whole = lm.grp > 0 || src != nullptr || epi != nullptr;
  const int chunk = (p2 && c->ntt_chunk > 0 && !whole) ? c->ntt_chunk : n_limbs;
  for (int off = 0; off < n_limbs; off += chunk) {
    const int cnt = n_limbs - off < chunk ? n_limbs - off : chunk;
    uint64_t* dc = d + (size_t)off * c->N;
    LimbMap lc = lm;
    lc.offset = lm.offset + off;
    if (!inverse) {
      launch_pass<false>(c, dc, cnt, lc, p1, 0, p2 == 0, src, p2 ? nullptr : epi);
      if (p2) launch_pass<false>(c, dc, cnt, lc, p2, p1, 1, nullptr, epi);
    } else {
      if (p2) {
        launch_pass<true>(c, dc, cnt, lc, p2, p1, 0, src);
        launch_pass<true>(c, dc, cnt, lc, p1, 0, 1);
      } else {
        launch_pass<true>(c, dc, cnt, lc, p1, 0, 1, src);
      }
    }
  }
}

}  // namespace lk
