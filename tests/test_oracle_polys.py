"""Pins for the oracle's polynomial tables against the paper's definitions."""
import os

import numpy as np
import pytest

from oracle import polys

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _balanced(p):
    return list(range(-(p - 1) // 2, (p - 1) // 2 + 1))


def test_lt0_truth_table_matches_table3():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "lt0_table3.txt")) if not ln.startswith("#")]
    assert rows
    for p, outs in rows:
        p = int(p)
        expect = [int(v) for v in outs.split(",")]
        c = polys.f_lt(p)
        got = [polys.eval_mod(c, x % p, p) for x in _balanced(p)]
        assert got == expect


def test_feq_values_match_eq2():
    for ln in open(os.path.join(GOLDEN, "feq_eq2.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        p, x, y, v = map(int, ln.split())
        assert polys.eval_mod(polys.f_eq(p), (x - y) % p, p) == v


@pytest.mark.parametrize("p", [3, 5, 13, 17, 257])
def test_flt_closed_form_is_the_sum_of_equality_polynomials(p):
    """F_LT0(x) = sum_{i=-(p-1)/2}^{-1} F_EQ(x, i) (Background, after Table 3), expanded by the
    binomial theorem and compared coefficient by coefficient with the closed form."""
    from math import comb
    acc = [0] * p
    for i in range(-(p - 1) // 2, 0):
        # 1 - (x - i)^(p-1) = 1 - sum_k C(p-1, k) x^k (-i)^(p-1-k)
        acc[0] = (acc[0] + 1) % p
        for k in range(p):
            acc[k] = (acc[k] - comb(p - 1, k) * pow(-i, p - 1 - k, p)) % p
    assert acc == polys.f_lt(p)
    # and the full truth table over Z_p
    for x in _balanced(p):
        assert polys.eval_mod(polys.f_lt(p), x % p, p) == (1 if x < 0 else 0)
        assert polys.eval_mod(polys.f_eq(p), x % p, p) == (1 if x == 0 else 0)


@pytest.mark.parametrize("p", [3, 5, 13, 17, 257])
def test_g_p2_satisfies_lemma3_on_all_of_z_p2(p):
    G = polys.g_p2(p)
    t = p * p
    assert len(G) - 1 <= (2 - 1) * (p - 1) + 1  # degree bound of Lemma 3
    # odd polynomial (parity property used for cheaper evaluation)
    assert all(c == 0 for c in G[0::2])
    xs = np.arange(t, dtype=np.int64)
    acc = np.zeros(t, dtype=np.int64)
    for c in reversed(G):
        acc = (acc * xs + c) % t
    z0 = ((xs + (p - 1) // 2) % p) - (p - 1) // 2  # balanced lowest digit
    assert np.array_equal(acc, z0 % t)


@pytest.mark.parametrize("p,e", [(3, 3), (5, 3), (5, 4), (5, 5), (7, 3), (7, 4), (13, 3), (17, 3)])
def test_g_pe_satisfies_lemma3_on_all_of_z_pe(p, e):
    """The lifted G_{p,e}: Lemma 3's property G(z0 + p z1) = z0 (mod p^e) on every element of
    Z_{p^e}, within Lemma 3's degree bound (e-1)(p-1)+1, odd."""
    G = polys.g_poly(p, e)
    t = p ** e
    assert len(G) - 1 <= (e - 1) * (p - 1) + 1
    assert all(c == 0 for c in G[0::2])
    assert all(0 <= c < t for c in G)
    xs = np.arange(t, dtype=np.int64)
    acc = np.zeros(t, dtype=np.int64)
    for c in reversed(G):
        acc = (acc * xs + c) % t
    z0 = ((xs + (p - 1) // 2) % p) - (p - 1) // 2
    assert np.array_equal(acc, z0 % t)


def test_g_pe_lift_needs_e_at_most_p():
    """The lift samples the error polynomial at e distinct points mod p."""
    with pytest.raises(ValueError):
        polys.g_poly(3, 4)
    assert polys.g_poly(5, 2) == polys.g_p2(5)
    assert polys.g_poly(7, 1) == [0, 1]


def test_g_p2_small_closed_forms():
    """Worked by hand: G_{3,2} = x^3 and G_{5,2} = x^5 + 20 x^3 + 5 x (mod 25).
    For p = 3: H interpolates (z - z^3)/3 = 0 at z in {-1, 0, 1}.  For p = 5: H
    interpolates (z - z^5)/5 at z = -2..2, i.e. values 6, 0, 0, 0, -6 = 1, 0, 0, 0, 4 mod 5,
    which is H = 4x^3 + x, so G = x^5 + 20x^3 + 5x."""
    assert polys.g_p2(3) == [0, 0, 0, 1]
    assert polys.g_p2(5) == [0, 5, 0, 20, 0, 1]


def test_lagrange_reproduces_a_known_polynomial():
    m = 17
    coeffs = [3, 0, 5, 16, 1]
    pts = list(range(5))
    vals = [polys.eval_mod(coeffs, x, m) for x in pts]
    assert polys.lagrange(pts, vals, m) == coeffs
