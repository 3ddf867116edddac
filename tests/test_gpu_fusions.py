"""The fused ModUp and ModDown give the same words as the separate launches they replace.

Key switching raises d2 to the special primes either inside the column pass of the forward
transform (bgv_set_modup_fused on, the default) or as inverse transform, basis extension and
forward transform in separate launches.  The two are compared on a two-pass ring small
enough for the oracle (whose parity tests run the fused form), at every first-pass length
the ring allows, and at the benchmark's ring (N = 2^16, 30 + 6 primes) with a broadcast
operand and with an operand that is a view of the lower limbs of a deeper batch.  The
product step's ModDown and switch (bgv_set_moddown_fused: 2 always fused, 0 separate) are
compared the same way: against the oracle on the two-pass ring, for every special-prime
count the kernel is built for and at the lowest levels a product step runs at (one and two
target rows), and at the benchmark's ring and the served mix's smaller rings at the batch
sizes where the default setting fuses."""
import numpy as np
import pytest
import torch

from oracle import bgv as B
from oracle import space as S
from tests.gpu_ctx import Pair, log, pair_two_pass

pytestmark = pytest.mark.gpu


def _both(lib, keys, a, b):
    f = lib.mul(keys, a, b)
    lib.set_modup_fused(False)
    try:
        u = lib.mul(keys, a, b)
    finally:
        lib.set_modup_fused(True)
    torch.cuda.synchronize()
    assert (f.n, f.level, f.t_exp, f.noise) == (u.n, u.level, u.t_exp, u.noise)
    w = f.n * lib.words(f.level)
    assert torch.equal(f.tensor[:w], u.tensor[:w]), "fused ModUp differs from the separate launches"
    return f


def test_fused_modup_matches_on_a_two_pass_ring():
    c = pair_two_pass()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(61)
    ga, oa = c.enc_both(g.integers(0, t, size=(3, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(3, P.ell)))
    try:
        for split in range(4, 7):  # every first-pass length the ring allows, so every second pass
            c.lib.set_ntt_split(split)
            f = _both(c.lib, c.keys, ga, gb)
            c.assert_equal(f, [S._mul(P, c.okeys, x, y) for x, y in zip(oa, ob)], f"product, split {split}")
    finally:
        c.lib.set_ntt_split(0)


def test_fused_modup_matches_at_the_benchmark_ring():
    log("[fusions] N=2^16 L=30 K=6")
    c = Pair(16, 257, 2, 30, 6, steps=(), conj=False, oracle_keys=False, hw=120)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(62)
    ga, _ = c.enc_both(g.integers(0, t, size=(3, P.ell)), oracle=False)
    gb, _ = c.enc_both(g.integers(0, t, size=(1, P.ell)), oracle=False)
    _both(c.lib, c.keys, ga, gb)  # broadcast b
    lo = c.lib.mod_switch_to(ga, 29)
    hi = c.lib.mul(c.keys, ga, ga)  # level 29: its noise lets lo's partner be dropped to 28
    _both(c.lib, c.keys, c.lib.mod_switch_to(lo, 28), hi)  # hi reaches 28 as a view of its limbs


def _both_moddown(lib, keys, a, b):
    try:
        lib.set_moddown_fused(2)  # fused whatever the batch
        f = lib.mul(keys, a, b)
        lib.set_moddown_fused(0)
        u = lib.mul(keys, a, b)
    finally:
        lib.set_moddown_fused(1)
    torch.cuda.synchronize()
    assert (f.n, f.level, f.t_exp, f.noise) == (u.n, u.level, u.t_exp, u.noise)
    w = f.n * lib.words(f.level)
    assert torch.equal(f.tensor[:w], u.tensor[:w]), "fused ModDown differs from the separate launches"
    return f


def test_fused_moddown_matches_on_a_two_pass_ring():
    """The product step's fused ModDown (last inverse pass of u's special and top rows, the
    merged correction and its first forward pass in one kernel) against the separate launches,
    at every first-pass length, and against the oracle."""
    c = pair_two_pass()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(63)
    ga, oa = c.enc_both(g.integers(0, t, size=(3, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(3, P.ell)))
    try:
        for split in range(4, 7):
            c.lib.set_ntt_split(split)
            f = _both_moddown(c.lib, c.keys, ga, gb)
            c.assert_equal(f, [S._mul(P, c.okeys, x, y) for x, y in zip(oa, ob)], f"product, split {split}")
    finally:
        c.lib.set_ntt_split(0)


def test_fused_moddown_matches_at_the_benchmark_ring():
    log("[fusions] ModDown N=2^16 L=30 K=6")
    c = Pair(16, 257, 2, 30, 6, steps=(), conj=False, oracle_keys=False, hw=120)
    P = c.P
    g = np.random.default_rng(64)
    ga, _ = c.enc_both(g.integers(0, P.t_full, size=(3, P.ell)), oracle=False)
    gb, _ = c.enc_both(g.integers(0, P.t_full, size=(1, P.ell)), oracle=False)
    _both_moddown(c.lib, c.keys, ga, gb)  # broadcast b
    lo = c.lib.mod_switch_to(ga, 25)  # a lower level: shorter chain of targets
    _both_moddown(c.lib, c.keys, lo, c.lib.mod_switch_to(ga, 25))
    # 16 ciphertexts: the default setting takes the fused kernel by itself
    gc, _ = c.enc_both(g.integers(0, P.t_full, size=(16, P.ell)), oracle=False)
    d = c.lib.mul(c.keys, gc, gc)
    f = _both_moddown(c.lib, c.keys, gc, gc)
    assert torch.equal(d.tensor[:f.n * c.lib.words(f.level)], f.tensor[:f.n * c.lib.words(f.level)])


@pytest.mark.parametrize("logN,L,K,n", [(14, 8, 2, 64), (15, 16, 4, 32)])
def test_fused_moddown_matches_on_the_served_rings(logN, L, K, n):
    """The served mix's smaller rings (7- and 8-stage first passes, K = 2 and 4) at the round sizes
    the server uses there, where the default setting takes the fused kernel."""
    log(f"[fusions] ModDown N=2^{logN} L={L} K={K} n={n}")
    c = Pair(logN, 257, 2, L, K, steps=(), conj=False, oracle_keys=False)
    g = np.random.default_rng(65 + logN)
    ga, _ = c.enc_both(g.integers(0, c.P.t_full, size=(n, c.P.ell)), oracle=False)
    gb, _ = c.enc_both(g.integers(0, c.P.t_full, size=(n, c.P.ell)), oracle=False)
    d = c.lib.mul(c.keys, ga, gb)
    f = _both_moddown(c.lib, c.keys, ga, gb)
    w = f.n * c.lib.words(f.level)
    assert torch.equal(d.tensor[:w], f.tensor[:w])


@pytest.mark.parametrize("K", [1, 3, 5, 6])
def test_fused_moddown_every_special_prime_count(K):
    """The special-prime counts the fused ModDown is built for beyond those above (K = 2 and 4), on
    a two-pass ring, against the separate launches and the oracle."""
    log(f"[fusions] ModDown N=2^10 L=8 K={K}")
    c = Pair(10, 17, 2, 8, K, steps=(), conj=False)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(70 + K)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    f = _both_moddown(c.lib, c.keys, ga, gb)
    c.assert_equal(f, [S._mul(P, c.okeys, x, y) for x, y in zip(oa, ob)], f"product, K = {K}")


@pytest.mark.parametrize("level", [2, 3])
def test_fused_moddown_at_the_lowest_levels(level):
    """The fused ModDown with one or two target rows (a product step at level 2 or 3), against
    the separate launches and the oracle."""
    c = pair_two_pass()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(80 + level)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    la, lb = c.lib.mod_switch_to(ga, level), c.lib.mod_switch_to(gb, level)
    ola = [B.align(P, x, level) for x in oa]
    olb = [B.align(P, x, level) for x in ob]
    f = _both_moddown(c.lib, c.keys, la, lb)
    c.assert_equal(f, [S._mul(P, c.okeys, x, y) for x, y in zip(ola, olb)], f"product at level {level}")
