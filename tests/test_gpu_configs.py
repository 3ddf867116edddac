"""Parity at the launch shapes of the primitive batch and of the ReLU workload.

Primitive batch: N = 2^15, p = 257, r = 2, 16 + 4 primes (digits of four), 64 ciphertexts per
call, as the benchmark's primitives leg runs them.  Two ciphertexts on each side alternate
through the batch (so an index mix-up between neighbours shows); mul_relin, rotation, the
modulus switch and both transforms are compared with the oracle at four batch positions, on
sampled coefficients for the ring products and on every word for the coefficient-wise switch.

ReLU: N = 2^16, 30 + 6 primes, 64 ciphertexts of int8 activations (the benchmark's ReLU call).
The oracle cannot run the 29-product pipeline at this ring size, so the checks are properties
that hold at any size: every activation decrypts to max(x, 0), and each ciphertext of the batched
call equals, word for word, the same ciphertext run alone.  The same schedule is compared with the
oracle word for word at N = 2^8 and 2^10 by test_gpu_parity_p257.py."""
import numpy as np
import pytest

from oracle import _ring as R
from oracle import bgv as B
from paper_2604_19890_amd import synth
from tests.gpu_ctx import Pair, log

pytestmark = pytest.mark.gpu


def test_primitive_batch_launch_shape_matches_the_oracle():
    log("[cfg] N=2^15 L=16 K=4, 64 ciphertexts")
    c = Pair(15, 257, 2, 16, 4, steps=(5,), conj=False, hw=120)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(15)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    A = c.lib.concat([c.lib.view(ga, i % 2, 1) for i in range(64)])
    Bt = c.lib.concat([c.lib.view(gb, (i + 1) % 2, 1) for i in range(64)])  # pairs (0,1), (1,0), ...
    idx = np.array([0, 1, 4097, P.N // 2 + 3, P.N - 1])
    positions = (0, 1, 62, 63)
    prod = c.lib.mul_relin(c.keys, A, Bt)
    rot = c.lib.rotate(c.keys, A, 5)
    sw = c.lib.mod_switch(A)
    wp, wr, ws = c.coeff_words(prod), c.coeff_words(rot), c.coeff_words(sw)
    for k in (0, 1):
        log(f"[cfg] oracle at sampled columns, pair {k} ...")
        ref_p = B.mul_relin_at(P, c.okeys.relin, oa[k], ob[1 - k], idx)
        ref_r = B.rotate_at(P, c.okeys.galois, oa[k], 5, idx)
        ref_s = B.mod_switch(P, oa[k]).c
        for pos in positions:
            if pos % 2 != k:
                continue
            assert np.array_equal(wp[pos][:, :, idx], ref_p), f"mul_relin at position {pos}"
            assert np.array_equal(wr[pos][:, :, idx], ref_r), f"rotate at position {pos}"
            assert np.array_equal(ws[pos], ref_s), f"mod_switch at position {pos}"
    # both transforms at the batch's shape (64 ciphertexts = 2048 limbs) on host-drawn coefficient
    # limbs: the forward outputs against the definition on sampled columns, then the round trip
    import torch
    rng = np.random.default_rng(1515)
    co = np.stack([rng.integers(0, q, size=(128, P.N), dtype=np.uint64) for q in P.primes[:P.L]], axis=1)
    x = torch.from_numpy(co.reshape(-1).view(np.int64).copy()).cuda()
    c.lib.ntt(x, 128, P.L, inverse=False)
    ev = x.cpu().numpy().view(np.uint64).reshape(128, P.L, P.N)
    for poly in (0, 1, 126, 127):
        for limb in (0, P.L - 1):
            q = P.primes[limb]
            assert np.array_equal(ev[poly, limb, idx], R.ntt_def_at(co[poly, limb], q, P.psi(q), idx)), (poly, limb)
    c.lib.ntt(x, 128, P.L, inverse=True)
    assert np.array_equal(x.cpu().numpy().view(np.uint64).reshape(co.shape), co), "round trip"
    # the products decrypt to the slot products
    ta, tb = c.lib.decrypt(c.s, ga).astype(object), c.lib.decrypt(c.s, gb).astype(object)
    got = c.lib.decrypt(c.s, prod)
    for pos in range(64):
        assert np.array_equal(got[pos], (ta[pos % 2] * tb[(pos + 1) % 2]) % t), pos


def test_relu_launch_shape_semantics_and_batch_equals_singles():
    from paper_2604_19890_amd import bgv as G
    log("[cfg] ReLU N=2^16 L=30 K=6, 64 ciphertexts")
    ctx = G.Context(16, 257, 2, 30, 6)
    s = synth.ternary(ctx.N, 0, 96)
    ka, ke = synth.key_randomness(ctx.primes, ctx.N, ctx.dnum, 0, 96, 0)
    keys = ctx.keygen(s, ka[None], ke[None])
    n = 64
    x = synth.int8_activations(n * ctx.slots, 32.0, 0, 96).reshape(n, ctx.slots)
    c1 = np.empty((n, ctx.L, ctx.N), dtype=np.uint64)
    e = np.empty((n, ctx.N), dtype=np.int32)
    for i in range(n):
        c1[i], e[i] = synth.encryption_randomness(ctx.primes[:ctx.L], ctx.N, 0, 96, i)
    X = ctx.encrypt(s, (x % ctx.t).astype(np.uint64), c1, e)
    out = ctx.relu(keys, X)
    got = ctx.decrypt(s, out)
    assert np.array_equal(got, np.maximum(x, 0) % ctx.t)
    assert (x < 0).any() and (x > 0).any()
    words = out.words(ctx.N)
    for pos in (0, 37, 63):
        single = ctx.relu(keys, ctx.view(X, pos, 1))
        assert (single.level, single.t_exp) == (out.level, out.t_exp)
        assert np.array_equal(single.words(ctx.N)[0], words[pos]), f"position {pos}"
