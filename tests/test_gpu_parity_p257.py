"""GPU parity of the headline circuit at the benchmark's plaintext modulus 257^2.

The benchmark's query runs p = 257, r = 2, 30 ciphertext primes and 6 special primes
(digits of six primes).  Those parameters take paths that no smaller prime reaches:
G_{257,2} and F_LT take the odd baby-step split with k = 32 (sixteen odd baby powers per
inner sum, nine inner sums at one level, eight outer products summed before one key
switch), F_EQ reuses F_LT's last giant power x^256, and the digits are balanced in
[-128, 128].  Here the whole circuit -- reduce (Algorithm 3), compare (Algorithm 4), raise
(the modulus-raising subsection), the masked product, the filter+SUM query and ReLU -- is
compared with the oracle ciphertext by ciphertext, word for word, at N = 2^8 (the one-pass
transform) and N = 2^10 (two passes and the fused key-switching pass), in both evaluation
schedules.  The slot values include the edges of the method: 0, +-1, the ends of the
centered range +-(p^2 - 1)/2, digits at +-(p - 1)/2 and carries between the digits."""
import functools

import numpy as np
import pytest

from oracle import bgv as B
from oracle import polys
from oracle import space as S
from tests.gpu_ctx import Pair, log, schedule

pytestmark = pytest.mark.gpu

P_, R_, L_, K_ = 257, 2, 30, 6
T_ = P_ ** R_
H_ = (T_ - 1) // 2  # 33024: the largest positive centered value
D_ = (P_ - 1) // 2  # 128: the largest balanced digit
ROT_STEPS = (1, 2, 4, 8, 16, 32)  # rotate-and-sum over a row of 64 slots


@functools.lru_cache(maxsize=None)
def pair257(log_n):
    return Pair(log_n, P_, R_, L_, K_, steps=ROT_STEPS, conj=True)


def edge_values():
    """Slot values at the edges of the method (mod 257^2)."""
    v = [0, 1, T_ - 1, 2, T_ - 2, H_, H_ + 1, H_ - 1, H_ + 2,
         D_, T_ - D_, D_ + 1, T_ - D_ - 1, P_, T_ - P_, P_ - 1, P_ + 1,
         D_ * P_, T_ - D_ * P_, D_ * P_ + D_, D_ * P_ - D_, T_ - (D_ * P_ - D_), (D_ + 1) * P_,
         D_ * P_ + D_ + 1, (D_ - 1) * P_ - D_]
    return [x % T_ for x in v]


def batch_rows(P, seed, n=3):
    """n rows of slot values: the first holds the edge values, the rest random ones."""
    g = np.random.default_rng(seed)
    rows = g.integers(0, T_, size=(n, P.ell)).tolist()
    e = edge_values()
    rows[0][:len(e)] = e
    return rows


def centered(v):
    v %= T_
    return v - T_ if v > H_ else v


def balanced_digits(v):
    z0 = v % P_
    z0 = z0 - P_ if z0 > D_ else z0
    z1 = ((v - z0) // P_) % P_
    return z0, z1


@pytest.mark.parametrize("sched", ["fast", "basic"])
def test_digit_and_lifting_polynomials_at_p257(sched):
    """eval_poly on G_{257,2} (t = 257^2) and F_LT, F_EQ (t = 257) against the oracle."""
    c = pair257(8)
    P = c.P
    ga, oa = c.enc_both(batch_rows(P, 1))
    with schedule(c, sched):
        g2 = polys.g_poly(P_, 2)
        c.assert_equal(c.lib.eval_poly(c.keys, ga, g2), [S.eval_poly(P, c.okeys, x, g2) for x in oa],
                       f"G_257,2 {sched}")
        gp = c.lib.set_t_exp(ga, 1)  # ChangeModToP: the slots become the values mod 257
        op = [B.change_mod_to_p(P, x) for x in oa]
        for name, cf in (("F_LT", polys.f_lt(P_)), ("F_EQ", polys.f_eq(P_))):
            c.assert_equal(c.lib.eval_poly(c.keys, gp, cf), [S.eval_poly(P, c.okeys, x, cf) for x in op],
                           f"{name} {sched}")


def _circuit(c, sched, seed):
    P = c.P
    rows = batch_rows(P, seed)
    v_rows = np.random.default_rng(seed + 100).integers(0, T_, size=(3, P.ell)).tolist()
    ga, oa = c.enc_both(rows)
    gv, ov = c.enc_both(v_rows)
    with schedule(c, sched):
        c.lib.reset_stats()
        gd = c.lib.space_reduce(c.keys, ga)
        glt = c.lib.compare(c.keys, gd, c.G.OP_LT)
        geq = c.lib.compare(c.keys, gd, c.G.OP_EQ)
        graise = c.lib.space_raise(c.keys, glt)
        gmask = c.lib.mul(c.keys, graise, gv)
        stats = c.lib.stats()
        log(f"[p257] N={P.N} {sched}: library done, stats {stats}; oracle ...")
        od = [S.space_reduce(P, c.okeys, x) for x in oa]
        for k in range(R_):
            c.assert_equal(gd[k], [d[k] for d in od], f"reduce digit {k} ({sched})")
        olt = [S.compare(P, c.okeys, d, "lt") for d in od]
        c.assert_equal(glt, olt, f"compare LT ({sched})")
        c.assert_equal(geq, [S.compare(P, c.okeys, d, "eq") for d in od], f"compare EQ ({sched})")
        oraise = [S.space_raise(P, c.okeys, x) for x in olt]
        c.assert_equal(graise, oraise, f"raise ({sched})")
        c.assert_equal(gmask, [S._mul(P, c.okeys, x, y) for x, y in zip(oraise, ov)], f"masked product ({sched})")
    # the semantics: balanced digits, centered LT, EQ with zero, raise of 0/1, v * LT
    dig = [c.lib.decrypt(c.s, d) for d in gd]
    lt = c.lib.decrypt(c.s, glt)
    eq = c.lib.decrypt(c.s, geq)
    rs = c.lib.decrypt(c.s, graise)
    mk = c.lib.decrypt(c.s, gmask)
    for b, row in enumerate(rows):
        for j, v in enumerate(row):
            z0, z1 = balanced_digits(v)
            assert (int(dig[0][b][j]), int(dig[1][b][j])) == (z0 % P_, z1 % P_), (b, j, v)
            want = 1 if centered(v) < 0 else 0
            assert int(lt[b][j]) == want and int(rs[b][j]) == want, (b, j, v)
            assert int(eq[b][j]) == (1 if v % T_ == 0 else 0), (b, j, v)
            assert int(mk[b][j]) == (v_rows[b][j] * want) % T_, (b, j, v)
    return stats


@pytest.mark.parametrize("log_n,sched", [(8, "fast"), (8, "basic"), (10, "fast"), (10, "basic")])
def test_headline_circuit_matches_at_p257(log_n, sched):
    """reduce -> compare (LT, EQ) -> raise -> multiply, three ciphertexts, both schedules."""
    stats = _circuit(pair257(log_n), sched, seed=log_n)
    if sched == "fast":
        # the launch shapes only p = 257 reaches: the odd split k = 32 of G_{257,2} and F_LT,
        # 16-term inner sums, all 9 inner sums of an evaluation in one pass, 8 outer pairs
        assert stats["max_baby_k"] == 32
        assert stats["max_inner_terms"] == 16
        assert stats["max_inner_outputs"] >= 9
        assert stats["max_tensor_pairs"] >= 8
        assert stats["limb_drops"] > 0 and stats["odd_splits"] >= 3
    else:
        assert stats["max_baby_k"] == 16 and stats["odd_splits"] == 0 and stats["limb_drops"] == 0


@pytest.mark.parametrize("log_n", [8, 10])
def test_filter_sum_and_relu_match_at_p257(log_n):
    """The query SUM(b * c WHERE a < thr) and ReLU at p = 257, the benchmark's schedule."""
    c = pair257(log_n)
    P = c.P
    g = np.random.default_rng(50 + log_n)
    thr = 40000
    a_rows = [[(thr + centered(v)) % T_ for v in row] for row in batch_rows(P, 60 + log_n)]  # a - thr at the edges
    b_rows = g.integers(0, 1 << 16, size=(3, P.ell)).tolist()
    c_rows = g.integers(0, 1 << 16, size=(3, P.ell)).tolist()
    ga, oa = c.enc_both(a_rows)
    gb, ob = c.enc_both(b_rows)
    gc, oc = c.enc_both(c_rows)
    gt, ot = c.enc_both([[thr] * P.ell])
    c.lib.reset_stats()
    fs = c.lib.filter_sum(c.keys, ga, gt, gb, gc)
    st = c.lib.stats()
    assert st["max_inner_terms"] == 16 and st["max_inner_outputs"] >= 9 and st["max_tensor_pairs"] >= 8
    log(f"[p257] N={P.N} filter_sum done; oracle ...")
    prods = [S.filter_product(P, c.okeys, x, ot[0], y, z) for x, y, z in zip(oa, ob, oc)]
    ref = S.rotate_and_sum(P, c.okeys, B.add_many(P, prods))
    c.assert_equal(fs, [ref], "filter_sum")
    want = sum(int(y) * int(z) for ra, rb, rc in zip(a_rows, b_rows, c_rows)
               for x, y, z in zip(ra, rb, rc) if centered(int(x) - thr) < 0) % T_
    assert np.array_equal(c.lib.decrypt(c.s, fs), np.array([[want] * P.ell]))
    # ReLU: x * (1 - [x < 0]) on values at the edges of the centered range
    x_rows = batch_rows(P, 70 + log_n)
    gx, ox = c.enc_both(x_rows)
    gr = c.lib.relu(c.keys, gx)
    c.assert_equal(gr, [S.relu(P, c.okeys, x) for x in ox], "relu")
    got = c.lib.decrypt(c.s, gr)
    for b, row in enumerate(x_rows):
        assert [int(v) for v in got[b]] == [v % T_ if centered(v) >= 0 else 0 for v in row], b


def test_sixteen_bit_query_exact_with_r3():
    """The 16-bit query with t = 257^3: every difference of two 16-bit values lies in the
    centered range of Z_{257^3}, so the circuit's predicate is the integer one.  Algorithm 3
    takes two G evaluations (G_{257,3} of degree 513, then G_{257,2}), Algorithm 4 aggregates
    three digits, and the raise is G_{257,3}; the chain needs 41 primes.  The filter products
    and the filter+SUM are compared with the oracle word for word at N = 2^8, and the SUM with
    the integer query."""
    c = Pair(8, P_, 3, 41, K_, steps=ROT_STEPS, conj=True)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(313)
    a_rows = g.integers(0, 1 << 16, size=(2, P.ell))
    a_rows[0][:6] = [0, 65535, 30000, 29999, 30001, 1]
    b_rows = g.integers(0, 1 << 16, size=(2, P.ell))
    c_rows = g.integers(0, 1 << 16, size=(2, P.ell))
    thr = 30000
    ga, oa = c.enc_both(a_rows)
    gb, ob = c.enc_both(b_rows)
    gc, oc = c.enc_both(c_rows)
    gt, ot = c.enc_both([[thr] * P.ell])
    log("[p257 r=3] N=2^8 L=41: library ...")
    fp = c.lib.filter_products(c.keys, ga, gt, gb, gc)
    fs = c.lib.filter_sum(c.keys, ga, gt, gb, gc)
    log("[p257 r=3] oracle ...")
    prods = [S.filter_product(P, c.okeys, x, ot[0], y, z) for x, y, z in zip(oa, ob, oc)]
    c.assert_equal(fp, prods, "filter products, r = 3")
    c.assert_equal(fs, [S.rotate_and_sum(P, c.okeys, B.add_many(P, prods))], "filter_sum, r = 3")
    want = int(sum(int(y) * int(z) for ra, rb, rc in zip(a_rows, b_rows, c_rows)
                   for x, y, z in zip(ra, rb, rc) if int(x) < thr) % t)
    assert np.array_equal(c.lib.decrypt(c.s, fs), np.array([[want] * P.ell]))
