"""GPU parity on extremal residues.

The kernels compute on residues below 2^50 as binary64 values with lazy reduction; the
bounds that keep this exact are checked on the host by test_arith_bounds.py.  Here the
kernels themselves run on words at the ends of the residue range -- every word q - 1,
alternating 0 and q - 1, every word (q - 1)/2, every word 1 -- and their results are
compared with the oracle: the NTT and its inverse against their definitions, and the
tensor product with relinearisation, the product step (relinearisation merged with a
modulus switch), rotation and repeated modulus switching against the oracle's ciphertext
operations.  Extremal words are not encryptions of anything; the operations are defined
on any words, and both sides compute the same function of them."""
import numpy as np
import pytest

from oracle import _ring as R
from oracle import bgv as B
from oracle import space as S
from oracle.params import Params
from tests.gpu_ctx import Pair, log, pair_two_pass

pytestmark = pytest.mark.gpu


def pattern(name, q, N):
    if name == "max":
        return np.full(N, q - 1, dtype=np.uint64)
    if name == "alternating":
        v = np.zeros(N, dtype=np.uint64)
        v[1::2] = q - 1
        return v
    if name == "half":
        return np.full(N, (q - 1) // 2, dtype=np.uint64)
    if name == "one":
        return np.ones(N, dtype=np.uint64)
    raise ValueError(name)


NAMES = ("max", "alternating", "half", "one")


def _upload(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint64).reshape(-1).view(np.int64).copy()).cuda()


def _download(t, shape):
    return t.cpu().numpy().view(np.uint64).reshape(shape)


def test_ntt_on_extremal_limbs_matches_the_definition_n1024():
    from paper_2604_19890_amd import bgv as G
    logN = 10
    lib = G.Context(logN, 17, 2, 3, 1)
    P = Params(logN, 17, 2, 3, 1)
    qs = P.primes[:4]
    x = np.stack([np.stack([pattern(nm, q, P.N) for q in qs]) for nm in NAMES])  # [4 patterns][4 primes][N]
    t = _upload(x)
    lib.ntt(t, len(NAMES), len(qs), inverse=False)
    got = _download(t, x.shape)
    for a, nm in enumerate(NAMES):
        for i, q in enumerate(qs):
            assert np.array_equal(got[a, i], R.ntt_def(x[a, i], q, P.psi(q))), (nm, i)
    # the same words as evaluation-form input of the inverse transform
    t = _upload(x)
    lib.ntt(t, len(NAMES), len(qs), inverse=True)
    got = _download(t, x.shape)
    for a, nm in enumerate(NAMES):
        for i, q in enumerate(qs):
            assert np.array_equal(got[a, i], R.intt_def(x[a, i], q, P.psi(q))), (nm, "inverse", i)


def test_ntt_on_extremal_limbs_n65536():
    """Forward transform of extremal coefficient vectors on sampled outputs; the inverse of
    constant evaluation vectors is the constant polynomial (closed form); round trips."""
    from paper_2604_19890_amd import bgv as G
    logN = 16
    lib = G.Context(logN, 257, 2, 3, 2)
    P = Params(logN, 257, 2, 3, 2)
    qs = P.primes[:5]
    x = np.stack([np.stack([pattern(nm, q, P.N) for q in qs]) for nm in NAMES])
    t = _upload(x)
    lib.ntt(t, len(NAMES), len(qs), inverse=False)
    got = _download(t, x.shape)
    idx = np.array([0, 1, 2, 3, 4097, P.N // 2 - 1, P.N // 2, P.N - 2, P.N - 1])
    for a, nm in enumerate(NAMES):
        for i, q in enumerate(qs):
            assert np.array_equal(got[a, i, idx], R.ntt_def_at(x[a, i], q, P.psi(q), idx)), (nm, i)
    lib.ntt(t, len(NAMES), len(qs), inverse=True)
    assert np.array_equal(_download(t, x.shape), x), "round trip"
    # constants in evaluation form (every word q - 1, (q - 1)/2 or 1) are the constant polynomials
    for nm in ("max", "half", "one"):
        c = np.stack([pattern(nm, q, P.N) for q in qs])
        t = _upload(c)
        lib.ntt(t, 1, len(qs), inverse=True)
        got = _download(t, c.shape)
        for i in range(len(qs)):
            want = np.zeros(P.N, dtype=np.uint64)
            want[0] = c[i, 0]
            assert np.array_equal(got[i], want), (nm, i)


def _extremal_pair(c, lv, names_a, names_b):
    """Ciphertext words built from patterns in evaluation form for the library, and their
    coefficient forms by the definition of the inverse transform for the oracle."""
    P = c.P
    qs = P.q[:lv]
    ev = np.zeros((2, 2, lv, P.N), dtype=np.uint64)
    co = np.zeros_like(ev)
    for k, names in enumerate((names_a, names_b)):
        for comp in range(2):
            for i, q in enumerate(qs):
                ev[k, comp, i] = pattern(names[comp], q, P.N)
                co[k, comp, i] = R.intt_def(ev[k, comp, i], q, P.psi(q))
    ga = c.lib.from_words(ev[0:1], P.r)
    gb = c.lib.from_words(ev[1:2], P.r)
    return ga, gb, B.Ct(co[0], lv, P.r), B.Ct(co[1], lv, P.r)


@pytest.mark.parametrize("names_a,names_b", [(("max", "max"), ("max", "max")),
                                             (("alternating", "max"), ("half", "alternating")),
                                             (("one", "half"), ("max", "one"))])
def test_products_rotation_and_switches_on_extremal_words_n1024(names_a, names_b):
    c = pair_two_pass()
    P = c.P
    ga, gb, oa, ob = _extremal_pair(c, P.L, names_a, names_b)
    c.assert_equal(c.lib.mul_relin(c.keys, ga, gb), [B.mul_relin(P, c.okeys.relin, oa, ob)], "mul_relin")
    c.assert_equal(c.lib.mul(c.keys, ga, gb), [S._mul(P, c.okeys, oa, ob)], "product step")
    c.lib.set_moddown_fused(2)  # the fused ModDown, which a single ciphertext does not take by default
    try:
        c.assert_equal(c.lib.mul(c.keys, ga, gb), [S._mul(P, c.okeys, oa, ob)], "product step, fused ModDown")
    finally:
        c.lib.set_moddown_fused(1)
    c.assert_equal(c.lib.rotate(c.keys, ga, 1), [B.rotate(P, c.okeys.galois, oa, 1)], "rotate")
    c.assert_equal(c.lib.mod_switch(gb), [B.mod_switch(P, ob)], "mod_switch")
    c.assert_equal(c.lib.mod_switch_to(ga, 1), [B.align(P, oa, 1)], "mod_switch_to 1")
    c.assert_equal(c.lib.add(ga, gb), [B.add(P, oa, ob)], "add")
    c.assert_equal(c.lib.sub(ga, gb), [B.sub(P, oa, ob)], "sub")


def test_product_step_on_extremal_words_at_the_benchmark_shape():
    """N = 2^16, 30 + 6 primes, level 30 (the fused key-switching pass at the benchmark's
    launch shape): extremal coefficient vectors, brought to evaluation form by the library's
    forward transform (checked against the definition above); the product step compared on
    sampled coefficients, repeated modulus switching on every word."""
    log("[extremes] N=2^16 L=30 K=6 level 30")
    c = Pair(16, 257, 2, 30, 6, steps=(), conj=False, hw=120)
    P = c.P
    lv = P.L
    co = np.zeros((2, 2, lv, P.N), dtype=np.uint64)
    for k, names in enumerate((("max", "alternating"), ("half", "max"))):
        for comp in range(2):
            for i, q in enumerate(P.q[:lv]):
                co[k, comp, i] = pattern(names[comp], q, P.N)
    t = _upload(co)
    c.lib.ntt(t, 4, lv, inverse=False)
    ev = _download(t, co.shape)
    ga = c.lib.from_words(ev[0:1], P.r)
    gb = c.lib.from_words(ev[1:2], P.r)
    oa, ob = B.Ct(co[0], lv, P.r), B.Ct(co[1], lv, P.r)
    idx = np.array([0, 1, 4097, P.N // 2 + 3, P.N - 1])
    prod = c.lib.mul(c.keys, ga, gb)
    log("[extremes] oracle product at sampled columns ...")
    ref = B.mul_relin_at(P, c.okeys.relin, oa, ob, idx)
    ref_ms = B.mod_switch_cols(P, B.Ct(ref, lv, P.r))
    assert np.array_equal(c.coeff_words(prod)[0][:, :, idx], ref_ms.c), "product step"
    c.lib.set_moddown_fused(2)
    try:
        prod_f = c.lib.mul(c.keys, ga, gb)
    finally:
        c.lib.set_moddown_fused(1)
    assert np.array_equal(c.coeff_words(prod_f)[0][:, :, idx], ref_ms.c), "product step, fused ModDown"
    c.assert_equal(c.lib.mod_switch_to(ga, 12), [B.align(P, oa, 12)], "mod_switch_to 12 (18 drops)")
    c.assert_equal(c.lib.mod_switch(gb), [B.mod_switch(P, ob)], "mod_switch")
