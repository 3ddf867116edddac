"""The allocation-free single modulus switch (bgv_mod_switch_noalloc) against the allocating
one (bgv_mod_switch, itself compared with the oracle elsewhere): bit for bit, on two calls in a
row with the second one smaller, on a second context of the same GPU (which shares the
scratch array), in place, and with a size above the scratch limit rejected on the host."""
import numpy as np
import pytest

from paper_2604_19890_amd import synth

pytestmark = pytest.mark.gpu

WL = 93


def _encrypt(ctx, n, seed):
    s = synth.ternary(ctx.N, seed, WL)
    g = np.random.default_rng(seed)
    slots = g.integers(0, ctx.t, size=(n, ctx.slots), dtype=np.uint64)
    c1 = np.empty((n, ctx.L, ctx.N), dtype=np.uint64)
    e = np.empty((n, ctx.N), dtype=np.int32)
    for i in range(n):
        c1[i], e[i] = synth.encryption_randomness(ctx.primes[:ctx.L], ctx.N, seed, WL, i)
    return ctx.encrypt(s, slots, c1, e)


def _same(ctx, x, y):
    assert (x.n, x.level, x.t_exp) == (y.n, y.level, y.t_exp)
    assert np.array_equal(x.words(ctx.N), y.words(ctx.N))


def test_noalloc_switch_equals_the_allocating_one():
    from paper_2604_19890_amd import bgv as G
    print("[noalloc] N=2^16 L=30 K=6", flush=True)
    big = G.Context(16, 257, 2, 30, 6)
    assert 2 * 1 * 30 * big.N <= G.NOALLOC_SCRATCH_WORDS < 2 * 2 * 30 * big.N
    a = _encrypt(big, 1, 1)
    # first call: the largest switch the scratch holds (one ciphertext at level 30)
    out = big.empty(1, 29)
    big.mod_switch_noalloc(a, out)
    _same(big, out, big.mod_switch(a))
    # second call, smaller: level 10 (the array keeps the first call's words beyond it)
    a10 = big.mod_switch_to(a, 10)
    out10 = big.empty(1, 9)
    big.mod_switch_noalloc(a10, out10)
    _same(big, out10, big.mod_switch(a10))
    # in place
    a11 = big.mod_switch_to(a, 11)
    ref = big.mod_switch(a11)
    big.mod_switch_noalloc(a11, a11)
    _same(big, a11, ref)
    # a batch above the limit is rejected before anything is enqueued; the output is untouched
    a2 = _encrypt(big, 2, 2)
    out2 = big.empty(2, 29)
    out2.tensor.fill_(7)
    with pytest.raises(G.BgvError) as ei:
        big.mod_switch_noalloc(a2, out2)
    assert ei.value.status == 1 and "scratch" in str(ei.value)
    big.sync()
    assert (out2.tensor == 7).all()


def test_noalloc_switch_on_a_second_context_of_the_gpu():
    """A batch of five on a small ring, after calls of a larger context on the same GPU."""
    from paper_2604_19890_amd import bgv as G
    small = G.Context(12, 17, 2, 18, 1)
    x = _encrypt(small, 5, 3)
    for lv in (18, 7):
        xl = small.mod_switch_to(x, lv)
        out = small.empty(5, lv - 1)
        small.mod_switch_noalloc(xl, out)
        _same(small, out, small.mod_switch(xl))
