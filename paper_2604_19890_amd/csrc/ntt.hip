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
#include "ntt_layout.hpp"
#include "ntt_stages.hpp"

namespace {

using namespace nttl;

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

void ntt_inverse_first_pass(bgv_ctx* c, uint64_t* d, const uint64_t* src, int n_limbs, LimbMap lm) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  launch_pass<true>(c, d, n_limbs, lm, p2, p1, 0, src);
}

void ntt_inverse_last_pass(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  launch_pass<true>(c, d, n_limbs, lm, p1, 0, 1);
}

void ntt_forward_last_pass(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm, const NttEpi* epi) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  launch_pass<false>(c, d, n_limbs, lm, p2, p1, 1, nullptr, epi);
}

void ntt_forward_first_pass(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm) {
  int p1, p2;
  ntt_split(c, &p1, &p2);
  launch_pass<false>(c, d, n_limbs, lm, p1, 0, 0);
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
