"""Pins for the oracle's polynomial evaluation and space-switching composites:
encrypted brute force over all of Z_{p^2} at tiny rings."""
import math

import numpy as np
import pytest

from oracle import bgv as B
from oracle import polys
from oracle import space as S
from tests.oracle_ctx import and5, p257, tiny5, tiny5_r3, tiny5_r4, tiny17, tiny37_r4


def _balanced_digits(v, p):
    h = (p - 1) // 2
    z0 = ((v + h) % p) - h
    z1 = ((v - z0) // p + h) % p - h
    return z0, z1


def _centered(v, m):
    v %= m
    return v - m if v > (m - 1) // 2 else v


@pytest.mark.parametrize("deg", [1, 2, 5, 16, 17, 31])
def test_bsgs_matches_horner_and_theorem2_depth(deg):
    c = tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(deg)
    coeffs = [int(x) for x in g.integers(0, t, size=deg + 1)]
    coeffs[deg] = coeffs[deg] or 1
    xs = [int(x) for x in g.integers(0, t, size=P.ell)]
    cnt = S.Counter()
    out = S.eval_poly(P, c.keys, c.enc(xs), coeffs, cnt)
    assert c.dec(out) == [polys.eval_mod(coeffs, x, t) for x in xs]
    depth = P.L - out.level
    assert depth <= math.ceil(math.log2(deg)) + 1 if deg > 1 else depth <= 1
    k, gg = S.bsgs_shape(deg)
    assert cnt.mul <= (k - 1) + (gg - 2) + (gg - 1)


@pytest.mark.parametrize("deg", [3, 5, 9, 17, 33])
def test_odd_split_matches_horner_and_is_no_deeper(deg):
    """Odd-structured polynomials (odd terms and a constant) take the odd split: the same
    plaintext values as Horner, depth within Theorem 2 and no deeper than the dense split."""
    c = tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(100 + deg)
    coeffs = [0] * (deg + 1)
    for i in range(1, deg + 1, 2):
        coeffs[i] = int(g.integers(1, t))
    coeffs[0] = int(g.integers(0, t))
    assert S.odd_structured(coeffs, deg)
    xs = [int(x) for x in g.integers(0, t, size=P.ell)]
    a = c.enc(xs)
    out = S.eval_poly(P, c.keys, a, coeffs)
    dense = S.eval_poly(P, c.keys, a, coeffs, parity=False)
    want = [polys.eval_mod(coeffs, x, t) for x in xs]
    assert c.dec(out) == want and c.dec(dense) == want
    assert P.L - out.level <= min(P.L - dense.level, math.ceil(math.log2(deg)) + 1)


def _products_needed(c, k, g):
    """Products a split needs when only the powers some term uses are formed: the power-rule
    closure of the used baby powers (and x^k), of the used giant powers, and one product per
    outer term whose inner sum is not a constant."""
    D = len(c) - 1
    coef = lambda n: c[n] if n <= D else 0

    def closure(need):
        need = set(need)
        for i in sorted(need, reverse=True):
            stack = [i]
            while stack:
                v = stack.pop()
                if v < 2:
                    continue
                h = 1 << (v.bit_length() - 1)
                parts = [v // 2] if v == h else [h, v - h]
                for q in parts:
                    if q not in need:
                        need.add(q)
                        stack.append(q)
        return {v for v in need if v >= 2}

    baby = closure([k] + [i for j in range(g) for i in range(1, k) if coef(j * k + i)])
    used_inner = [any(coef(j * k + i) for i in range(1, k)) for j in range(g)]
    giant = closure([j for j in range(1, g) if used_inner[j] or coef(j * k)])
    outer = sum(1 for j in range(1, g) if used_inner[j])
    return len(baby) + len(giant) + outer


def test_odd_split_of_the_space_switching_polynomials():
    """G_{p,2} (odd) and F_LT (odd terms and x^(p-1)) take the odd split, which keeps the
    dense split's depth of 9 at p = 257 and cuts the products it needs:
    - G: 20 baby (x^2, x^4, .., x^32 and the odd x^3..x^31) + 7 giant + 8 outer = 35, against
      11 + 15 + 16 = 42 with k = 16;
    - F_LT: 19 baby (it vanishes at every 17 + 32j, so x^17 is never formed) + 7 giant + 7
      outer (x^256 enters as a scalar multiple of the last giant power) = 33, against
      11 + 15 + 15 = 41.
    x^(p-1) stays the last giant power, which the comparison reuses for EQ."""
    for p, shape in ((17, (8, 3)), (257, (32, 9))):
        t = p * p
        G = [v % t for v in polys.g_poly(p, 2)]
        F = [v % p for v in polys.f_lt(p)]
        for poly in (G, F):
            D = len(poly) - 1
            assert S.odd_structured(poly, D)
            assert S.bsgs_shape(D, True) == shape
        k, g = shape
        assert (g - 1) * k == p - 1
    G = [v % 66049 for v in polys.g_poly(257, 2)]
    F = [v % 257 for v in polys.f_lt(257)]
    assert _products_needed(G, *S.bsgs_shape(257, True)) == 35
    assert _products_needed(G, *S.bsgs_shape(257)) == 42
    assert all(F[17 + 32 * j] == 0 for j in range(8))
    assert _products_needed(F, *S.bsgs_shape(256, True)) == 33
    assert _products_needed(F, *S.bsgs_shape(256)) == 41


@pytest.mark.parametrize("ctx", [tiny5, tiny17])
def test_space_reduce_brute_force(ctx):
    c = ctx()
    P, p, t = c.P, c.P.p, c.P.t_full
    for start in range(0, t, P.ell):
        vals = [(start + i) % t for i in range(P.ell)]
        dg = S.space_reduce(P, c.keys, c.enc(vals))
        assert [d.t_exp for d in dg] == [1, 1]
        got0, got1 = c.dec(dg[0]), c.dec(dg[1])
        for v, a0, a1 in zip(vals, got0, got1):
            z0, z1 = _balanced_digits(v, p)
            assert (a0, a1) == (z0 % p, z1 % p)


@pytest.mark.parametrize("ctx", [tiny5, tiny17])
def test_compare_brute_force(ctx):
    """LT and EQ of every d in Z_{p^2} against zero: LT = [centered(d) < 0], EQ = [d = 0]."""
    c = ctx()
    P, p, t = c.P, c.P.p, c.P.t_full
    step = P.ell if P.ell > 2 else 2
    for start in range(0, t, step):
        vals = [(start + i) % t for i in range(P.ell)]
        dg = S.space_reduce(P, c.keys, c.enc(vals))
        lt = c.dec(S.compare(P, c.keys, dg, "lt"))
        eq = c.dec(S.compare(P, c.keys, dg, "eq"))
        assert lt == [1 if _centered(v, t) < 0 else 0 for v in vals]
        assert eq == [1 if v == 0 else 0 for v in vals]


@pytest.mark.parametrize("ctx", [tiny5, tiny17])
def test_predicate_family_brute_force(ctx):
    """GT, GE, LE and NEQ (the comparison subsection's family) for every d in Z_{p^2}."""
    c = ctx()
    P, p, t = c.P, c.P.p, c.P.t_full
    ref = {"gt": lambda v: _centered(v, t) > 0, "ge": lambda v: _centered(v, t) >= 0,
           "le": lambda v: _centered(v, t) <= 0, "neq": lambda v: v % t != 0}
    step = P.ell if P.ell > 2 else 2
    for start in range(0, t, step * (3 if t > 100 else 1)):
        vals = [(start + i) % t for i in range(P.ell)]
        dg = S.space_reduce(P, c.keys, c.enc(vals))
        for op, f in ref.items():
            assert c.dec(S.compare(P, c.keys, dg, op)) == [1 if f(v) else 0 for v in vals], op


def _balanced_digits_r(v, p, r):
    h = (p - 1) // 2
    out = []
    for _ in range(r):
        z = ((v + h) % p) - h
        out.append(z)
        v = (v - z) // p
    return out


def test_space_reduce_r3_brute_force():
    """Algorithm 3 with r = 3 (G_{5,3}, then G_{5,2}): the three balanced base-5 digits of
    every value of Z_125."""
    c = tiny5_r3()
    P, p, t = c.P, c.P.p, c.P.t_full
    assert t == 125
    for start in range(0, t, P.ell):
        vals = [(start + i) % t for i in range(P.ell)]
        dg = S.space_reduce(P, c.keys, c.enc(vals))
        assert [d.t_exp for d in dg] == [1, 1, 1]
        got = [c.dec(d) for d in dg]
        for k, v in enumerate(vals):
            assert [g[k] for g in got] == [z % p for z in _balanced_digits_r(v, p, 3)]


def test_compare_and_raise_r3_brute_force():
    """r = 3: LT and EQ of every d in Z_125 against zero through three digits, and raise of the
    LT result back to Z_125 (G_{5,3})."""
    c = tiny5_r3()
    P, p, t = c.P, c.P.p, c.P.t_full
    for start in range(0, t, P.ell):
        vals = [(start + i) % t for i in range(P.ell)]
        dg = S.space_reduce(P, c.keys, c.enc(vals))
        lt = S.compare(P, c.keys, dg, "lt")
        assert c.dec(lt) == [1 if _centered(v, t) < 0 else 0 for v in vals]
        assert c.dec(S.compare(P, c.keys, dg, "eq")) == [1 if v == 0 else 0 for v in vals]
        up = S.space_raise(P, c.keys, lt)
        assert up.t_exp == 3
        assert c.dec(up) == [1 if _centered(v, t) < 0 else 0 for v in vals]


@pytest.mark.parametrize("ctx,vals", [
    (tiny5_r4, [0, 1, 2, 3, 312, 313, 314, 622, 623, 624, 100, 500]),
    (tiny37_r4, [0, 1874160, 937080, 937081]),  # t = 37^4 = 1874161: 0, -1, and both sides of the middle
])
def test_space_switching_r4_sampled(ctx, vals):
    """r = 4 (Table 6's r): the four balanced digits, LT against zero and its raise, on values
    around zero, around the middle of Z_{p^4} and elsewhere."""
    c = ctx()
    P, p, t = c.P, c.P.p, c.P.t_full
    for i in range(0, len(vals), P.ell):
        v = (vals[i:i + P.ell] + vals[:P.ell])[:P.ell]
        dg = S.space_reduce(P, c.keys, c.enc(v))
        got = [c.dec(d) for d in dg]
        for k, x in enumerate(v):
            assert [g[k] for g in got] == [z % p for z in _balanced_digits_r(x, p, 4)]
        lt = S.compare(P, c.keys, dg, "lt")
        assert c.dec(lt) == [1 if _centered(x, t) < 0 else 0 for x in v]
        assert c.dec(S.space_raise(P, c.keys, lt)) == [1 if _centered(x, t) < 0 else 0 for x in v]


def test_fgt_truth_table():
    for p in (5, 17, 257):
        for x in range(-(p - 1) // 2, (p - 1) // 2 + 1):
            assert polys.eval_mod(polys.f_gt(p), x % p, p) == (1 if x > 0 else 0)


@pytest.mark.parametrize("ctx", [tiny5, tiny17])
def test_space_raise_clears_high_digits(ctx):
    """Raise of k + p*junk (tagged p) returns centered_p(k) mod p^2."""
    c = ctx()
    P, p, t = c.P, c.P.p, c.P.t_full
    g = np.random.default_rng(11)
    for _ in range(3):
        ks = [int(x) for x in g.integers(0, p, size=P.ell)]
        junk = [int(x) for x in g.integers(0, p, size=P.ell)]
        ct = B.change_mod_to_p(P, c.enc([(k + p * j) % t for k, j in zip(ks, junk)]))
        out = S.space_raise(P, c.keys, ct)
        assert out.t_exp == P.r
        assert c.dec(out) == [_centered(k, p) % t for k in ks]


def test_masked_product_pipeline_small_p():
    """v * [x < y] through reduce -> compare -> raise -> multiply (all pairs for p = 5)."""
    c = tiny5()
    P, p, t = c.P, c.P.p, c.P.t_full
    pairs = [(x, y) for x in range(p) for y in range(p)]
    for i in range(0, len(pairs), P.ell):
        chunk = pairs[i:i + P.ell]
        chunk += [(0, 0)] * (P.ell - len(chunk))
        xs = [a for a, _ in chunk]
        ys = [b for _, b in chunk]
        vs = [(3 * a + b + 1) % t for a, b in chunk]
        out = S.masked_product(P, c.keys, c.enc(xs), c.enc(ys), c.enc(vs))
        assert out.level >= 1
        assert c.dec(out) == [v if a < b else 0 for v, a, b in zip(vs, xs, ys)]


def test_relu_and_filter_sum_pipelines():
    c = tiny17()
    P, t = c.P, c.P.t_full
    xs = [-100, -1, 0, 1, 17, 144, -144, 55]
    out = S.relu(P, c.keys, c.enc([x % t for x in xs]))
    assert out.level >= 1
    assert c.dec(out) == [max(x, 0) % t for x in xs]
    a = [3, 90, 200, 4, 16, 1, 2, 150]
    b = [5, 6, 7, 8, 9, 10, 11, 12]
    cc = [2, 3, 4, 5, 6, 7, 8, 9]
    thr = 100
    prod = S.filter_product(P, c.keys, c.enc(a), c.enc([thr] * P.ell), c.enc(b), c.enc(cc))
    assert c.dec(prod) == [(x * y if v < thr else 0) % t for v, x, y in zip(a, b, cc)]
    total = S.rotate_and_sum(P, c.keys, prod)
    expect = sum(x * y for v, x, y in zip(a, b, cc) if v < thr) % t
    assert c.dec(total) == [expect] * P.ell


def _basic_products(c, k, g):
    """Products of the basic schedule: every baby power x^2..x^k, every giant power
    y^2..y^(g-1), and one product per j >= 1 whose inner sum is not a constant."""
    D = len(c) - 1
    coef = lambda n: c[n] if n <= D else 0
    outer = sum(1 for j in range(1, g) if any(coef(j * k + i) for i in range(1, k)))
    return (k - 1) + (g - 2) + outer


def test_basic_schedule_counts_horner_and_depth():
    """The basic schedule (dense split, own-level inner sums, one product per outer term) on
    encrypted inputs: Horner's values, the products counted by hand and the fast schedule's
    depth.  G_{17,2} (D = 17, k = 4, g = 5): 3 baby + 3 giant + 4 outer = 10; a dense degree-16
    polynomial: 3 + 3 + 3 = 9 (its I_4 is the constant c_16).  At p = 257 the same count gives
    15 + 15 + 16 = 46 for G_{257,2} and 15 + 15 + 15 = 45 for F_LT (x^256 enters as a scalar
    multiple of y^16)."""
    c = tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(7)
    G = [v % t for v in polys.g_poly(17, 2)]
    dense16 = [int(v) for v in g.integers(1, t, size=17)]
    xs = [int(x) for x in g.integers(0, t, size=P.ell)]
    a = c.enc(xs)
    try:
        for poly, want in ((G, 10), (dense16, 9)):
            P.schedule = "basic"
            cnt = S.Counter()
            out = S.eval_poly(P, c.keys, a, poly, cnt)
            assert c.dec(out) == [polys.eval_mod(poly, x, t) for x in xs]
            assert cnt.mul == want == _basic_products(poly, *S.bsgs_shape(len(poly) - 1))
            P.schedule = "fast"
            fast = S.eval_poly(P, c.keys, a, poly)
            assert out.level == fast.level
    finally:
        P.schedule = "fast"
    G257 = [v % 66049 for v in polys.g_poly(257, 2)]
    F257 = [v % 257 for v in polys.f_lt(257)]
    assert S.bsgs_shape(257) == (16, 17) and S.bsgs_shape(256) == (16, 17)
    assert _basic_products(G257, 16, 17) == 46
    assert _basic_products(F257, 16, 17) == 45


def test_basic_schedule_space_switching_brute_force():
    """reduce -> LT -> raise in the basic schedule over all of Z_25 (p = 5): the same plaintext
    results as the fast schedule (centered x < 0)."""
    c = tiny5()
    P, t = c.P, c.P.t_full
    vals = list(range(t))
    try:
        P.schedule = "basic"
        got = []
        for s0 in range(0, t, P.ell):
            chunk = (vals[s0:s0 + P.ell] + [0] * P.ell)[:P.ell]
            digits = S.space_reduce(P, c.keys, c.enc(chunk))
            got += c.dec(S.space_raise(P, c.keys, S.compare(P, c.keys, digits, "lt")))[: len(vals[s0:s0 + P.ell])]
    finally:
        P.schedule = "fast"
    assert got == [1 if v > (t - 1) // 2 else 0 for v in vals]


def _p257_edges(t, p):
    h, d = (t - 1) // 2, (p - 1) // 2
    v = [0, 1, t - 1, 2, t - 2, h, h + 1, h - 1, h + 2, d, t - d, d + 1, t - d - 1, p, t - p, p - 1, p + 1,
         d * p, t - d * p, d * p + d, d * p - d, (d + 1) * p, d * p + d + 1, (d - 1) * p - d]
    return [x % t for x in v]


@pytest.mark.parametrize("sched", ["fast", "basic"])
def test_space_switching_at_p257_encrypted(sched):
    """The benchmark's modulus 257^2 (30 + 6 primes, N = 2^8): one ciphertext whose 128 slots
    hold the edges of the method (0, +-1, +-(t-1)/2, digits at +-(p-1)/2, carries between the
    digits) and random values.  The decrypted digits are the balanced base-p digits (Lemma 3),
    LT is [centered value < 0], EQ is [value = 0], and the raise is the 0/1 lift (plain
    definitions, not the circuit)."""
    c = p257()
    P, t, p = c.P, c.P.t_full, c.P.p
    vals = _p257_edges(t, p)
    vals += [int(x) for x in np.random.default_rng(257).integers(0, t, size=P.ell - len(vals))]
    P.schedule = sched
    try:
        dg = S.space_reduce(P, c.keys, c.enc(vals))
        lt = S.compare(P, c.keys, dg, "lt")
        eq = S.compare(P, c.keys, dg, "eq")
        rs = S.space_raise(P, c.keys, lt)
    finally:
        P.schedule = "fast"
    assert [d.t_exp for d in dg] == [1, 1] and rs.t_exp == 2
    got0, got1 = c.dec(dg[0]), c.dec(dg[1])
    want = [_balanced_digits(v, p) for v in vals]
    assert got0 == [z0 % p for z0, _ in want]
    assert got1 == [z1 % p for _, z1 in want]
    assert all(z0 + p * z1 == _centered(v, t) for v, (z0, z1) in zip(vals, want))
    lt_want = [1 if _centered(v, t) < 0 else 0 for v in vals]
    assert c.dec(lt) == lt_want
    assert c.dec(eq) == [1 if v == 0 else 0 for v in vals]
    assert c.dec(rs) == lt_want


@pytest.mark.parametrize("preds_kind", ["range", "two_columns", "three"])
def test_filter_conjunction_brute_force(preds_kind):
    """The conjunction of predicates (range filters) against its plain definition over Z_{p^2},
    p = 5: every slot of the result is b * c when every predicate holds on the centered values,
    else 0; the predicates of the comparison subsection (LT, GE, LE, NEQ, EQ)."""
    c = and5()
    P, t, ell = c.P, c.P.t_full, c.P.ell
    g = np.random.default_rng(len(preds_kind))
    cen = lambda v: _centered(v, t)
    rel = {"lt": lambda x, y: cen(x - y) < 0, "ge": lambda x, y: cen(x - y) >= 0, "le": lambda x, y: cen(x - y) <= 0,
           "gt": lambda x, y: cen(x - y) > 0, "eq": lambda x, y: (x - y) % t == 0, "neq": lambda x, y: (x - y) % t != 0}
    a = [int(v) for v in g.integers(0, t, size=ell)]
    d = [int(v) for v in g.integers(0, t, size=ell)]
    bv = [int(v) for v in g.integers(0, t, size=ell)]
    cv = [int(v) for v in g.integers(0, t, size=ell)]
    if preds_kind == "range":      # lo <= a < hi
        spec = [(a, 3, "ge"), (a, 15, "lt")]
    elif preds_kind == "two_columns":
        spec = [(a, 10, "le"), (d, 7, "neq")]
    else:
        spec = [(a, 20, "lt"), (d, 0, "ge"), (a, 2, "neq")]
    enc_cols = {id(a): c.enc(a), id(d): c.enc(d)}
    preds = [(enc_cols[id(col)], c.enc([thr] * ell), op) for col, thr, op in spec]
    cnt = S.Counter()
    out = S.filter_and_product(P, c.keys, preds, c.enc(bv), c.enc(cv), cnt)
    want = [(bv[j] * cv[j]) % t if all(rel[op](col[j], thr) for col, thr, op in spec) else 0 for j in range(ell)]
    assert c.dec(out) == want
    assert out.level >= 1
