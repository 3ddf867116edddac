"""GPU parity of the multi-predicate filter SUM(b*c WHERE pred_0 AND pred_1 ..) against the oracle,
word for word: p = 17 with two and three predicates over two columns, and the benchmark's modulus
257^2 with a range predicate (lo <= a < hi) on a 31-prime chain (the single-predicate query's 30
plus one level for the conjunction)."""
import functools

import numpy as np
import pytest

from oracle import bgv as B
from oracle import space as S
from tests.gpu_ctx import Pair, log

pytestmark = pytest.mark.gpu

OPS = {"lt": 0, "eq": 1, "gt": 2, "le": 3, "ge": 4, "neq": 5}


@functools.lru_cache(maxsize=None)
def pair_and17():
    return Pair(5, 17, 2, 20, 1, steps=(1, 2), conj=True)


@functools.lru_cache(maxsize=None)
def pair_and257():
    return Pair(8, 257, 2, 31, 6, steps=(1, 2, 4, 8, 16, 32), conj=True)


def _run(c, spec, n, seed, sum_too):
    """spec: list of (column name, threshold, op); columns drawn per name."""
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(seed)
    names = sorted({s[0] for s in spec})
    rows = {nm: g.integers(0, t, size=(n, P.ell)) for nm in names}
    enc = {nm: c.enc_both(rows[nm]) for nm in names}
    gb, ob = c.enc_both(g.integers(0, t, size=(n, P.ell)))
    gc, oc = c.enc_both(g.integers(0, t, size=(n, P.ell)))
    thr = [c.enc_both([[th] * P.ell]) for _, th, _ in spec]
    gpreds = [(enc[nm][0], thr[i][0], OPS[op]) for i, (nm, th, op) in enumerate(spec)]
    prods = c.lib.filter_and_products(c.keys, gpreds, gb, gc)
    log(f"[and] N={P.N} p={P.p} {len(spec)} predicates: oracle ...")
    oprods = [S.filter_and_product(P, c.okeys, [(enc[nm][1][b], thr[i][1][0], op) for i, (nm, th, op) in enumerate(spec)],
                                   ob[b], oc[b]) for b in range(n)]
    c.assert_equal(prods, oprods, "filter_and_products")
    cen = lambda v: v - t if v > (t - 1) // 2 else v
    rel = {"lt": lambda x, y: cen((x - y) % t) < 0, "ge": lambda x, y: cen((x - y) % t) >= 0,
           "le": lambda x, y: cen((x - y) % t) <= 0, "neq": lambda x, y: (x - y) % t != 0}
    got = c.lib.decrypt(c.s, prods)
    bv, cv = c.lib.decrypt(c.s, gb), c.lib.decrypt(c.s, gc)
    for b in range(n):
        for j in range(P.ell):
            ok = all(rel[op](int(rows[nm][b][j]), th) for nm, th, op in spec)
            assert int(got[b][j]) == ((int(bv[b][j]) * int(cv[b][j])) % t if ok else 0), (b, j)
    if sum_too:
        fs = c.lib.filter_and_sum(c.keys, gpreds, gb, gc)
        c.assert_equal(fs, [S.rotate_and_sum(P, c.okeys, B.add_many(P, oprods))], "filter_and_sum")


@pytest.mark.parametrize("spec", [[("a", 40, "ge"), ("a", 200, "lt")],
                                  [("a", 150, "le"), ("d", 17, "neq"), ("d", 100, "lt")]])
def test_conjunction_matches_at_p17(spec):
    _run(pair_and17(), spec, 3, len(spec), sum_too=True)


def test_range_filter_matches_at_p257():
    c = pair_and257()
    _run(c, [("a", 1000, "ge"), ("a", 40000, "lt")], 2, 257, sum_too=False)
