// Host check of the library's binary64 modular arithmetic (modarith.hpp) and of the
// lazy-reduction bounds of its butterfly stages (ntt_stages.hpp), on adversarial and
// random operands, against exact 128-bit integer arithmetic.  Built with g++ by
// tests/test_arith_bounds.py; prints one JSON object per modulus.
//
// Checked for each modulus q in [2^49, 2^50) given on the command line:
//   mul_lazy: for |a| <= m q and 0 <= b < q, the result is congruent to a b and its
//     magnitude is at most (3 m / 8 + 1/2) q (m = 1, 1.9, 3.1, 4.8, 8);
//   red: for |x| < 2^53 the result is congruent to x and at most q/2 + 1 in magnitude;
//   ct_stages<D>: from |v| <= q, after 1..4 Cooley-Tukey stages every value is congruent
//     to the exact butterfly network's and below 1.9, 3.1, 4.8, 7.1 q;
//   gs_stages<D>: from |v| <= q, after 1..4 Gentleman-Sande stages every value is
//     congruent to the exact network's and below 4 q, every multiplicand below 8 q;
//   split accumulation: 16 terms x < q with integer coefficients |c| < 2^24 give
//     hi, lo exact and split_combine congruent to sum c x.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "modarith.hpp"
#include "ntt_stages.hpp"

typedef __int128 i128;

static int failures = 0;

static void fail(const char* what, double q, double a, double b, double r) {
  if (failures < 20) std::fprintf(stderr, "FAIL %s q=%.0f a=%.17g b=%.17g r=%.17g\n", what, q, a, b, r);
  ++failures;
}

static int64_t as_int(double x) { return (int64_t)x; }
static bool integral(double x) { return std::floor(x) == x && std::fabs(x) < 9007199254740992.0; }

static i128 mod(i128 x, i128 q) {
  i128 r = x % q;
  return r < 0 ? r + q : r;
}

int main(int argc, char** argv) {
  std::mt19937_64 rng(12345);
  for (int ai = 1; ai < argc; ++ai) {
    const uint64_t qi = std::strtoull(argv[ai], nullptr, 10);
    const double q = (double)qi, qinv = 1.0 / q;
    auto urand = [&](double lo, double hi) {
      std::uniform_real_distribution<double> d(lo, hi);
      return std::nearbyint(d(rng));
    };
    // ---- mul_lazy
    const double ms[5] = {1.0, 1.9, 3.1, 4.8, 8.0};
    double mul_max[5] = {0, 0, 0, 0, 0};
    for (int mi = 0; mi < 5; ++mi) {
      const double m = ms[mi];
      const double amax = std::floor(m * q);
      std::vector<double> as = {0, 1, -1, q - 1, -(q - 1), q, -q, amax, -amax, amax - 1, -(amax - 1),
                                std::floor((q - 1) / 2), std::floor((q + 1) / 2), std::floor(amax / 2)};
      std::vector<double> bs = {0, 1, q - 1, q - 2, std::floor((q - 1) / 2), std::floor((q + 1) / 2),
                                std::floor(q / 3), std::floor(2 * q / 3)};
      for (int k = 0; k < 60000; ++k) {
        double a, b;
        if (k < (int)(as.size() * bs.size())) {
          a = as[k / bs.size()];
          b = bs[k % bs.size()];
        } else {
          a = urand(-amax, amax);
          b = urand(0, q - 1);
        }
        const double r = mul_lazy(a, b, q, qinv);
        if (!integral(r) || mod((i128)as_int(r) - (i128)as_int(a) * (i128)as_int(b), qi) != 0)
          fail("mul_lazy congruence", q, a, b, r);
        const double ratio = std::fabs(r) / q;
        if (ratio > mul_max[mi]) mul_max[mi] = ratio;
        if (ratio > 3.0 * m / 8.0 + 0.5) fail("mul_lazy bound", q, a, b, r);
      }
    }
    // ---- red
    double red_max = 0;
    for (int k = 0; k < 60000; ++k) {
      double x;
      const double lim = 9007199254740991.0;  // 2^53 - 1
      if (k < 8) {
        const double xs[8] = {lim, -lim, lim - 1, -(lim - 1), q, -q, 0, 4503599627370495.0};
        x = xs[k];
      } else {
        x = urand(-lim, lim);
      }
      const double r = red(x, q, qinv);
      if (!integral(r) || mod((i128)as_int(r) - (i128)as_int(x), qi) != 0) fail("red congruence", q, x, 0, r);
      if (std::fabs(r) > red_max) red_max = std::fabs(r);
      if (std::fabs(r) > q / 2 + 1) fail("red bound", q, x, 0, r);
    }
    // ---- butterfly stages on 16 registers (N = 16, g0 = 0, gs_log = 0: twiddles w[1..15])
    double ct_max[4] = {0, 0, 0, 0}, gs_max[4] = {0, 0, 0, 0};
    double gs_mult_max = 0;
    for (int trial = 0; trial < 20000; ++trial) {
      double v0[16], w[16];
      const int mode = trial % 6;
      for (int i = 0; i < 16; ++i) {
        switch (mode) {
          case 0: v0[i] = (i & 1) ? q : -q; break;
          case 1: v0[i] = q; break;
          case 2: v0[i] = ((trial >> (i % 8)) & 1) ? q - 1 : -(q - 1); break;
          default: v0[i] = urand(-q, q); break;
        }
        w[i] = (mode == 1 || (mode == 2 && (i & 1))) ? q - 1 : urand(0, q - 1);
      }
      for (int depth = 1; depth <= 4; ++depth) {
        // ct_stages<D> runs the stages at distances D, D/2, .., 1, so the magnitudes after
        // the first `depth` stages of the four-stage step come from a stage-by-stage replay
        // with the same operations (checked against ct_stages<8> below)
        double v[16];
        for (int i = 0; i < 16; ++i) v[i] = v0[i];
        i128 e[16];
        for (int i = 0; i < 16; ++i) e[i] = mod((i128)as_int(v0[i]), qi);
        int dd = 8;
        for (int s = 0; s < depth; ++s, dd >>= 1) {
          // one Cooley-Tukey stage at distance dd with the same twiddle indexing
          const double* wp = w + (16 >> (__builtin_ctz(2 * dd)));
          for (int g = 0; g < 16 / (2 * dd); ++g) {
            const double wt = wp[g];
            for (int i = g * 2 * dd; i < g * 2 * dd + dd; ++i) {
              const double r = mul_lazy(v[i + dd], wt, q, qinv);
              const double a = v[i];
              v[i] = a + r;
              v[i + dd] = a - r;
              const i128 t = mod(e[i + dd] * (i128)as_int(wt), qi);
              const i128 x = e[i];
              e[i] = mod(x + t, qi);
              e[i + dd] = mod(x - t, qi);
            }
          }
        }
        for (int i = 0; i < 16; ++i) {
          if (!integral(v[i]) || mod((i128)as_int(v[i]), qi) != e[i]) fail("ct stage congruence", q, v0[i], w[1], v[i]);
          ct_max[depth - 1] = std::fmax(ct_max[depth - 1], std::fabs(v[i]) / q);
        }
        if (depth == 4) {
          double lib[16];
          for (int i = 0; i < 16; ++i) lib[i] = v0[i];
          ct_stages<8>(lib, w, 16, 0, 0, q, qinv);
          for (int i = 0; i < 16; ++i)
            if (lib[i] != v[i]) fail("ct_stages<8> differs from its stage-by-stage replay", q, v0[i], w[1], lib[i]);
        }
      }
      // the full 4-stage step as the kernels run it, against the exact network
      {
        double v[16];
        for (int i = 0; i < 16; ++i) v[i] = v0[i];
        ct_stages<8>(v, w, 16, 0, 0, q, qinv);
        i128 e[16];
        for (int i = 0; i < 16; ++i) e[i] = mod((i128)as_int(v0[i]), qi);
        for (int dd = 8; dd >= 1; dd >>= 1) {
          const double* wp = w + (16 >> (__builtin_ctz(2 * dd)));
          for (int g = 0; g < 16 / (2 * dd); ++g)
            for (int i = g * 2 * dd; i < g * 2 * dd + dd; ++i) {
              const i128 t = mod(e[i + dd] * (i128)as_int(wp[g]), qi);
              const i128 x = e[i];
              e[i] = mod(x + t, qi);
              e[i + dd] = mod(x - t, qi);
            }
        }
        for (int i = 0; i < 16; ++i) {
          if (!integral(v[i]) || mod((i128)as_int(v[i]), qi) != e[i]) fail("ct_stages<8>", q, v0[i], w[1], v[i]);
          if (std::fabs(v[i]) >= 7.1 * q) fail("ct_stages<8> bound", q, v0[i], w[1], v[i]);
        }
      }
      {
        double v[16];
        for (int i = 0; i < 16; ++i) v[i] = v0[i];
        gs_stages<8>(v, w, 16, 0, 0, q, qinv);
        i128 e[16];
        for (int i = 0; i < 16; ++i) e[i] = mod((i128)as_int(v0[i]), qi);
        // stage by stage: track magnitudes with the same operations as gs_stages
        double u[16];
        for (int i = 0; i < 16; ++i) u[i] = v0[i];
        int stage = 0;
        for (int dd = 1; dd <= 8; dd <<= 1) {
          ++stage;
          const double* wp = w + (16 >> (__builtin_ctz(2 * dd)));
          for (int g = 0; g < 16 / (2 * dd); ++g) {
            const double wt = wp[g];
            for (int i = g * 2 * dd; i < g * 2 * dd + dd; ++i) {
              const double a = u[i], b = u[i + dd];
              gs_mult_max = std::fmax(gs_mult_max, std::fabs(a - b) / q);
              const double s = a + b;
              u[i] = (stage & 1) ? s : red(s, q, qinv);
              u[i + dd] = mul_lazy(a - b, wt, q, qinv);
              const i128 x = e[i], y = e[i + dd];
              e[i] = mod(x + y, qi);
              e[i + dd] = mod((x - y) * (i128)as_int(wt), qi);
            }
          }
          for (int i = 0; i < 16; ++i) gs_max[stage - 1] = std::fmax(gs_max[stage - 1], std::fabs(u[i]) / q);
        }
        for (int i = 0; i < 16; ++i) {
          if (v[i] != u[i]) fail("gs_stages<8> differs from its stage-by-stage replay", q, v0[i], w[1], v[i]);
          if (!integral(v[i]) || mod((i128)as_int(v[i]), qi) != e[i]) fail("gs_stages<8>", q, v0[i], w[1], v[i]);
          if (std::fabs(v[i]) >= 4.0 * q) fail("gs_stages<8> bound", q, v0[i], w[1], v[i]);
        }
      }
    }
    if (gs_mult_max >= 8.0) fail("gs multiplicand bound", q, gs_mult_max, 0, 0);
    // ---- split accumulation of small-coefficient linear combinations
    const int64_t cmax = (1 << 24) - 1;
    for (int trial = 0; trial < 20000; ++trial) {
      double hi = 0, lo = 0;
      i128 exact = 0;
      for (int t = 0; t < 16; ++t) {
        uint64_t x;
        int64_t c;
        if (trial < 4) {
          x = qi - 1;
          c = (trial & 1) ? cmax : (((t + trial / 2) & 1) ? cmax : -cmax);
        } else {
          x = rng() % qi;
          c = (int64_t)(rng() % (2 * cmax + 1)) - cmax;
        }
        hi = __builtin_fma((double)c, split_hi(x), hi);
        lo = __builtin_fma((double)c, split_lo(x), lo);
        exact += (i128)c * (i128)x;
      }
      if (!integral(hi) || !integral(lo)) fail("split sums not exact", q, hi, lo, 0);
      const double r = split_combine(hi, lo, q, qinv);
      if (!integral(r) || mod((i128)as_int(r) - exact, qi) != 0) fail("split_combine congruence", q, hi, lo, r);
      if (std::fabs(r) >= 2 * q) fail("split_combine bound", q, hi, lo, r);
    }
    std::printf(
        "{\"q\": %llu, \"mul_max\": [%.4f, %.4f, %.4f, %.4f, %.4f], \"red_max_over_q\": %.6f, "
        "\"ct_max\": [%.4f, %.4f, %.4f, %.4f], \"gs_max\": [%.4f, %.4f, %.4f, %.4f], \"gs_mult_max\": %.4f, "
        "\"failures\": %d}\n",
        (unsigned long long)qi, mul_max[0], mul_max[1], mul_max[2], mul_max[3], mul_max[4], red_max / q, ct_max[0],
        ct_max[1], ct_max[2], ct_max[3], gs_max[0], gs_max[1], gs_max[2], gs_max[3], gs_mult_max, failures);
  }
  return failures == 0 ? 0 : 1;
}
