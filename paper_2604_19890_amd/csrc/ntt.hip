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
#include "ctx.hpp"

namespace {

constexpr int NT_MAX = 256;

__device__ __forceinline__ int lds_idx(int sl, int k, int S) { return sl * (S + (S >> 4) + 1) + k + (k >> 4); }

template <int LOGS, bool INV>
__global__ void __launch_bounds__(NT_MAX) k_ntt_pass(uint64_t* __restrict__ data, int logN, int s0, LimbMap lm,
                                                     const PrimeD* __restrict__ pc,
                                                     const double* __restrict__ tw, int first, int last) {
  constexpr int S = 1 << LOGS;
  constexpr int T = S / 16;
  __shared__ double lds[NT_MAX * 16 + NT_MAX + NT_MAX];
  const int N = 1 << logN;
  const int NT = blockDim.x;
  const int SUBS = NT / T;
  const int limb = blockIdx.y;
  if (limb_skipped(lm, limb)) return;
  const int pi = limb_prime(lm, limb);
  const double q = pc[pi].q, qinv = pc[pi].qinv;
  const double* __restrict__ w = tw + (size_t)pi * N;
  uint64_t* __restrict__ x = data + (size_t)limb * N;
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
  const int st = blockIdx.x * SUBS + sl;
  const int lo = st & (tmin - 1);
  const int hi = st >> tmin_log;
  const int base = (hi << (tmax_log + 1)) + lo;
  double v[16];

  // load in the coalesced order: k = tau + T*i
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = u2d(x[base + (tau + T * i) * tmin]);

  if (!INV) {
    // stages with local half-distance 8T, 4T, 2T, T (register distance 8, 4, 2, 1)
#pragma unroll
    for (int dd = 8; dd >= 1; dd >>= 1) {
      const int tg_log = tmin_log + __builtin_ctz(dd * T);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (i & dd) continue;
        const int jup = base + (tau + T * i) * tmin;
        const double wt = w[(N + jup) >> (tg_log + 1)];
        const double r = mul_lazy(v[i + dd], wt, q, qinv);
        const double a = v[i];
        v[i] = red(a + r, q, qinv);
        v[i + dd] = red(a - r, q, qinv);
      }
    }
    if (T > 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = v[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
      // remaining stages: local half-distance T/2 .. 1 on consecutive points
#pragma unroll
      for (int dd = 8; dd >= 1; dd >>= 1) {
        if (dd >= T) continue;
        const int tg_log = tmin_log + __builtin_ctz(dd);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          if (i & dd) continue;
          const int jup = base + (16 * tau + i) * tmin;
          const double wt = w[(N + jup) >> (tg_log + 1)];
          const double r = mul_lazy(v[i + dd], wt, q, qinv);
          const double a = v[i];
          v[i] = red(a + r, q, qinv);
          v[i + dd] = red(a - r, q, qinv);
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = v[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
    }
  } else {
    if (T > 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, tau + T * i, S)] = v[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, 16 * tau + i, S)];
#pragma unroll
      for (int dd = 1; dd <= 8; dd <<= 1) {
        if (dd >= T) continue;
        const int tg_log = tmin_log + __builtin_ctz(dd);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          if (i & dd) continue;
          const int jup = base + (16 * tau + i) * tmin;
          const double wt = w[(N + jup) >> (tg_log + 1)];
          const double a = v[i], b = v[i + dd];
          v[i] = red(a + b, q, qinv);
          v[i + dd] = mul_lazy(red(a - b, q, qinv), wt, q, qinv);
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[lds_idx(sl, 16 * tau + i, S)] = v[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = lds[lds_idx(sl, tau + T * i, S)];
    }
#pragma unroll
    for (int dd = 1; dd <= 8; dd <<= 1) {
      const int tg_log = tmin_log + __builtin_ctz(dd * T);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (i & dd) continue;
        const int jup = base + (tau + T * i) * tmin;
        const double wt = w[(N + jup) >> (tg_log + 1)];
        const double a = v[i], b = v[i + dd];
        v[i] = red(a + b, q, qinv);
        v[i + dd] = mul_lazy(red(a - b, q, qinv), wt, q, qinv);
      }
    }
    if (last) {
      const double ninv = pc[pi].ninv;
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = mul_lazy(v[i], ninv, q, qinv);
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) x[base + (tau + T * i) * tmin] = d2u(canon(red(v[i], q, qinv), q));
  (void)first;
}

template <bool INV>
void launch_pass(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm, int logS, int s0, int first, int last) {
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
    hipLaunchKernelGGL((k_ntt_pass<LS, INV>), grid, dim3(NT), 0, c->stream, d, c->logN, s0, lm, c->d_prime, \
                       tw, first, last);                                                                   \
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

void ntt(bgv_ctx* c, uint64_t* d, int n_limbs, LimbMap lm, bool inverse) {
  if (n_limbs <= 0) return;
  const int logN = c->logN;
  int p1, p2;
  if (logN <= 8) {
    p1 = logN;
    p2 = 0;
  } else {
    p1 = (logN + 1) / 2;
    p2 = logN - p1;
  }
  if (!inverse) {
    launch_pass<false>(c, d, n_limbs, lm, p1, 0, 1, p2 == 0);
    if (p2) launch_pass<false>(c, d, n_limbs, lm, p2, p1, 0, 1);
  } else {
    if (p2) {
      launch_pass<true>(c, d, n_limbs, lm, p2, p1, 1, 0);
      launch_pass<true>(c, d, n_limbs, lm, p1, 0, 0, 1);
    } else {
      launch_pass<true>(c, d, n_limbs, lm, p1, 0, 1, 1);
    }
  }
}

}  // namespace lk
