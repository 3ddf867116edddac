"""Pins of the oracle's noise estimate (oracle/noise.py).

The estimate is a bound, so it is pinned against what it bounds: the measured noise
max |[c0 + c1 s]_Q| of every ciphertext the oracle produces through whole pipelines
(reduce, compare, raise, the filter product, rotate-and-sum, ReLU) must stay below
2^(nz/16), in both schedules and at several (p, r).  A dropped or mis-scaled term in
the model (a missing sqrt(N) in the tensor bound, a switch floor without t) shows
up there as a measured noise above its estimate.  The integer helpers are pinned
against exact arithmetic."""
import math

import numpy as np
import pytest

from oracle import bgv as B
from oracle import noise as NZ
from oracle import space as S
from tests.oracle_ctx import Ctx


def p257():
    """The benchmark's plaintext modulus 257^2 and chain on N = 2^8, with the rotation keys of
    rotate-and-sum."""
    global _P257
    if _P257 is None:
        _P257 = Ctx(8, 257, 2, 30, 6, steps=(1, 2, 4, 8, 16, 32), conj=True)
    return _P257


_P257 = None

pytestmark = pytest.mark.timeout(900)


def test_fixed_point_logs_are_exact():
    for x in list(range(1, 5000)) + [2 ** 31 - 1, 2 ** 32, 3 ** 20, 257 ** 2, 20 * 66049, (1 << 50) - 27]:
        c, f = NZ.lgc(x), NZ.lgf(x)
        v = 16 * math.log2(x)
        assert f <= v + 1e-9 and c >= v - 1e-9, x
        assert c - f in (0, 1) and (c == f) == (x & (x - 1) == 0 and round(v) == v), x
        # exact: 2^f <= x^16 <= 2^c, with f largest and c smallest
        assert 2 ** f <= x ** 16 <= 2 ** c
        assert x ** 16 < 2 ** (f + 1) and (c == 0 or x ** 16 > 2 ** (c - 1))


def test_lsum_bounds_the_sum_of_the_bounds():
    for a in range(0, 900, 7):
        for d in range(0, 200):
            b = a + d
            exact = 16 * math.log2(2 ** (a / 16) + 2 ** (b / 16))
            assert NZ.lsum(a, b) >= exact - 1e-9 and NZ.lsum(b, a) == NZ.lsum(a, b), (a, b)
    assert NZ.lsum(100, 100) == 116  # equal bounds: one bit more


def test_sum_of_n_bounds_n_terms():
    for a in (1, 7, 100, 333, 800):
        for n in list(range(1, 70)) + [255, 256, 257, 8192, 10 ** 6]:
            e = NZ.sum_of(a, n)
            assert e >= a + 16 * math.log2(n) - 1e-9 and e - (a + 16 * math.log2(n)) < 1, (a, n)
            assert 2 ** e >= n ** 16 * 2 ** a  # exact: n 2^(a/16) <= 2^(e/16)
    assert NZ.sum_of(0, 5) == 0  # unknown stays unknown
    # against the chain of pairwise sums: equal for two and three terms, tighter from four on
    for a in (50, 400):
        chain = a
        for n in range(2, 300):
            chain = NZ.add(chain, a)
            if n <= 3:
                assert NZ.sum_of(a, n) == chain, n
            else:
                assert NZ.sum_of(a, n) < chain, n


def test_sum_estimate_bounds_the_noise_of_long_sums():
    """The n-term bound against the measured noise of sums of fresh ciphertexts and of
    products, at the benchmark's plaintext modulus."""
    c = p257()
    P = c.P
    rng = np.random.default_rng(15)
    fresh = [c.enc(rng.integers(0, P.t_full, P.ell)) for _ in range(40)]
    for n in (4, 17, 40):
        tot = B.add_many(P, fresh[:n])
        assert _measured_bits(P, c.s, tot) <= tot.nz / 16
    prods = [S._mul(P, c.keys, fresh[i], fresh[i + 1]) for i in range(0, 16, 2)]
    tot = B.add_many(P, prods)
    assert _measured_bits(P, c.s, tot) <= tot.nz / 16
    assert _measured_bits(P, c.s, S.rotate_and_sum(P, c.keys, tot)) <= S.rotate_and_sum(P, c.keys, tot).nz / 16


def _measured_bits(P, s, ct):
    V = B.phase(P, s, ct)
    mx = max(abs(v) for v in V)
    return math.log2(mx) if mx else 0.0


class _Recorder:
    """Records every ciphertext the oracle's operations return during a pipeline."""

    NAMES = ("add", "sub", "neg", "mul_scalar", "add_const", "divide_by_p", "change_mod_to_p", "raise_tag",
             "mod_switch", "drop", "relin", "rotate")

    def __init__(self, monkeypatch):
        self.cts = []
        for name in self.NAMES:
            f = getattr(B, name)

            def wrap(*a, _f=f, _name=name, **k):
                r = _f(*a, **k)
                self.cts.append((_name, r))
                return r

            monkeypatch.setattr(B, name, wrap)


def _check_bounds(c, rec, limit=None):
    """Every recorded ciphertext: measured noise <= estimate; returns the smallest slack seen."""
    worst = 1e9
    seen = 0
    # the ciphertexts are many and their phases cost a CRT each: check a spread of them
    step = max(1, len(rec.cts) // (limit or len(rec.cts)))
    for name, ct in rec.cts[::step]:
        assert NZ.known(ct.nz), name
        got = _measured_bits(c.P, c.s, ct)
        slack = ct.nz / 16 - got
        assert slack >= 0, f"{name}: measured {got:.2f} bits above the estimate {ct.nz / 16:.2f} (level {ct.level}, t_exp {ct.t_exp})"
        worst = min(worst, slack)
        seen += 1
    assert seen > 0
    return worst


def _query(c, rng, thr=None):
    P, t = c.P, c.P.t_full
    a = c.enc(rng.integers(0, t, P.ell))
    th = c.enc([thr if thr is not None else int(rng.integers(0, t))] * P.ell)
    b = c.enc(rng.integers(0, t, P.ell))
    cc = c.enc(rng.integers(0, t, P.ell))
    return a, th, b, cc


def test_fresh_estimate_bounds_fresh_noise():
    c = p257()
    rng = np.random.default_rng(3)
    for _ in range(4):
        ct = c.enc(rng.integers(0, c.P.t_full, c.P.ell))
        assert ct.nz == NZ.model(c.P).fresh
        assert _measured_bits(c.P, c.s, ct) <= ct.nz / 16


@pytest.mark.parametrize("schedule", ["fast", "basic"])
def test_estimate_bounds_the_noise_through_the_query_at_p257(monkeypatch, schedule):
    c = p257()
    c.P.schedule = schedule
    try:
        rng = np.random.default_rng(11)
        a, th, b, cc = _query(c, rng, thr=1000)
        rec = _Recorder(monkeypatch)
        pr = S.filter_product(c.P, c.keys, a, th, b, cc)
        tot = S.rotate_and_sum(c.P, c.keys, pr)
        slack = _check_bounds(c, rec, limit=120)
        assert tot.level >= 1
        # the final value's measured noise leaves room below q_0 / 2
        assert _measured_bits(c.P, c.s, tot) < math.log2(c.P.q[0]) - 1 - 10
        assert slack < 8  # the bound is not vacuous
    finally:
        c.P.schedule = "fast"


def test_estimate_bounds_the_noise_through_relu_at_p257(monkeypatch):
    c = p257()
    rng = np.random.default_rng(12)
    x = c.enc([int(v) % c.P.t_full for v in rng.integers(-100, 100, c.P.ell)])
    rec = _Recorder(monkeypatch)
    lt = S.less_than(c.P, c.keys, x, None)
    S._mul(c.P, c.keys, x, B.add_const(c.P, B.neg(c.P, lt), 1))
    _check_bounds(c, rec, limit=80)


@pytest.mark.parametrize("args", [(4, 5, 3, 17, 1), (5, 17, 2, 18, 1), (4, 5, 2, 14, 1)])
def test_estimate_bounds_the_noise_on_small_rings(monkeypatch, args):
    c = Ctx(*args)
    rng = np.random.default_rng(13)
    a, th, b, cc = _query(c, rng)
    rec = _Recorder(monkeypatch)
    S.filter_product(c.P, c.keys, a, th, b, cc)
    for op in ("lt", "gt", "eq", "neq"):
        S.compare(c.P, c.keys, S.space_reduce(c.P, c.keys, B.sub(c.P, a, th)), op)
    _check_bounds(c, rec)


def test_fast_schedule_lowers_mostly_by_dropping(monkeypatch):
    """The query at p = 257 takes few rescaling switches beyond its products in the fast
    schedule, against hundreds of single-prime alignments in the basic one (the estimate
    pins above show the noise stays bounded either way)."""
    c = p257()
    rng = np.random.default_rng(14)
    a, th, b, cc = _query(c, rng, thr=1000)
    counts = {}
    for schedule in ("fast", "basic"):
        c.P.schedule = schedule
        f_ms = B.mod_switch
        lowered = []

        def count_ms(P, x, _f=f_ms):
            lowered.append(1)
            return _f(P, x)

        monkeypatch.setattr(B, "mod_switch", count_ms)
        try:
            S.filter_product(c.P, c.keys, a, th, b, cc)
        finally:
            c.P.schedule = "fast"
            monkeypatch.setattr(B, "mod_switch", f_ms)
        counts[schedule] = len(lowered)
    # one switch per product in both; the basic schedule adds one per level of every alignment
    assert counts["basic"] > 3 * counts["fast"], counts
