"""GPU parity on rings with the two-pass NTT (and the fused key-switching pass), the tiny
workload end to end at N = 4096, and sampled checks at the real sizes N = 2^15 and 2^16."""
import math

import numpy as np
import pytest

from oracle import bgv as B
from oracle import space as S
from tests.gpu_ctx import Pair, log, pair_two_pass, schedule

pytestmark = pytest.mark.gpu


def test_two_pass_ring_operations_match():
    c = pair_two_pass()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(21)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    c.assert_equal(c.lib.mul_relin(c.keys, ga, gb), [B.mul_relin(P, c.okeys.relin, x, y) for x, y in zip(oa, ob)],
                   "mul_relin N=1024")
    om = [S._mul(P, c.okeys, x, y) for x, y in zip(oa, ob)]
    for split in (4, 6, 0):  # the fused key-switching pass under every pass split
        c.lib.set_ntt_split(split)
        c.assert_equal(c.lib.mul(c.keys, ga, gb), om, f"mul N=1024 split {split}")
    c.assert_equal(c.lib.rotate(c.keys, ga, 1), [B.rotate(P, c.okeys.galois, x, 1) for x in oa], "rotate N=1024")
    c.assert_equal(c.lib.rotate(c.keys, ga, c.G.ROW_SWAP), [B.rotate(P, c.okeys.galois, x, "conj") for x in oa],
                   "conj N=1024")
    c.assert_equal(c.lib.mod_switch_to(ga, 2), [B.align(P, x, 2) for x in oa], "mod_switch_to N=1024")
    coeffs = [int(v) for v in g.integers(0, t, size=6)]
    c.assert_equal(c.lib.eval_poly(c.keys, ga, coeffs), [S.eval_poly(P, c.okeys, x, coeffs) for x in oa],
                   "eval_poly N=1024")


def test_products_on_a_ring_with_a_four_stage_second_pass():
    """N = 2^9: the default pass split is 5 + 4, so the fused pass has a single register step."""
    c = Pair(9, 17, 2, 5, 2)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(23)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    c.assert_equal(c.lib.mul_relin(c.keys, ga, gb), [B.mul_relin(P, c.okeys.relin, x, y) for x, y in zip(oa, ob)],
                   "mul_relin N=512")
    c.assert_equal(c.lib.mul(c.keys, ga, gb), [S._mul(P, c.okeys, x, y) for x, y in zip(oa, ob)], "mul N=512")


def test_tiny_workload_end_to_end_n4096():
    """v * [x < y] with N = 4096, p = 17, 18 primes + 1 special prime: every word of the result."""
    c = Pair(12, 17, 2, 18, 1)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(0)
    xs, ys, vs = (g.integers(0, 17, size=(1, P.ell)) for _ in range(3))
    gx, ox = c.enc_both(xs)
    gy, oy = c.enc_both(ys)
    gv, ov = c.enc_both(vs)
    lt = c.lib.less_than(c.keys, gx, gy)
    out = c.lib.mul(c.keys, lt, gv)
    log("[e2e] oracle pipeline at N=4096 ...")
    ref = S.masked_product(P, c.okeys, ox[0], oy[0], ov[0])
    c.assert_equal(out, [ref], "masked product N=4096")
    expect = [int(v) if a < b else 0 for v, a, b in zip(vs[0], xs[0], ys[0])]
    assert list(c.lib.decrypt(c.s, out)[0]) == expect
    assert out.level >= 1


def _sampled_words(c, gct, idx):
    w = c.coeff_words(gct)
    return w[:, :, :, idx]


@pytest.mark.parametrize("shape", [(15, 257, 2, 16, 4, 16), (16, 257, 2, 30, 6, 8)])
def test_full_size_products_sampled(shape):
    """mul_relin, the product step and a rotation at N = 2^15 (L = 16, K = 4) and N = 2^16
    (L = 30, K = 6, taken at a lower level), compared on sampled coefficients.  The secret has
    Hamming weight 120 (the paper's parameter) so that the oracle's key generation stays fast."""
    logN, p, r, L, K, lv = shape
    log(f"[full] logN={logN} L={L} K={K} level={lv}")
    c = Pair(logN, p, r, L, K, steps=(1,), conj=False, hw=120)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(logN)
    ga, oa = c.enc_both(g.integers(0, t, size=(1, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(1, P.ell)))
    idx = np.array([0, 1, 4097, P.N // 2 + 3, P.N - 1])
    # encryption on sampled columns
    assert np.array_equal(_sampled_words(c, ga, idx)[0], B.sampled(P, oa[0], idx).c)
    if lv < L:
        ga, gb = c.lib.mod_switch_to(ga, lv), c.lib.mod_switch_to(gb, lv)
        oa = [B.align(P, oa[0], lv)]
        ob = [B.align(P, ob[0], lv)]
        assert np.array_equal(_sampled_words(c, ga, idx)[0], B.sampled(P, oa[0], idx).c)
    log("[full] oracle mul_relin at sampled columns ...")
    ref = B.mul_relin_at(P, c.okeys.relin, oa[0], ob[0], idx)
    got = c.lib.mul_relin(c.keys, ga, gb)
    assert np.array_equal(_sampled_words(c, got, idx)[0], ref), "mul_relin"
    prod = c.lib.mul(c.keys, ga, gb)
    ref_ms = B.mod_switch_cols(P, B.Ct(ref, lv, oa[0].t_exp))
    assert np.array_equal(_sampled_words(c, prod, idx)[0], ref_ms.c), "product step (merged switch)"
    rot = c.lib.rotate(c.keys, ga, 1)
    assert np.array_equal(_sampled_words(c, rot, idx)[0], B.rotate_at(P, c.okeys.galois, oa[0], 1, idx)), "rotate"
    # and the semantics at full size
    ta, tb = c.lib.decrypt(c.s, ga)[0], c.lib.decrypt(c.s, gb)[0]
    assert np.array_equal(c.lib.decrypt(c.s, prod)[0], (ta.astype(object) * tb.astype(object)) % t)


def test_full_size_batch_in_the_bench_launch_shape():
    """The product step on a batch of 32 ciphertexts at the top of the N = 2^16, L = 30, K = 6
    chain, the launch shape the benchmark times.  Two ciphertext pairs alternate through the
    batch, so an index mix-up between neighbours shows; four positions are compared with the
    oracle on sampled coefficients."""
    log("[batch32] N=2^16 L=30 K=6, 32 ciphertexts at level 30")
    c = Pair(16, 257, 2, 30, 6, steps=(), conj=False, hw=120)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(32)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    A = c.lib.concat([c.lib.view(ga, i % 2, 1) for i in range(32)])
    Bt = c.lib.concat([c.lib.view(gb, i % 2, 1) for i in range(32)])
    prod = c.lib.mul(c.keys, A, Bt)
    assert prod.n == 32 and prod.level == P.L - 1
    idx = np.array([0, 1, 4097, P.N // 2 + 3, P.N - 1])
    for k in (0, 1):
        log(f"[batch32] oracle product of pair {k} at sampled columns ...")
        ref = B.mul_relin_at(P, c.okeys.relin, oa[k], ob[k], idx)
        ref_ms = B.mod_switch_cols(P, B.Ct(ref, P.L, oa[k].t_exp))
        for pos in (k, 30 + k):
            got = _sampled_words(c, c.lib.view(prod, pos, 1), idx)[0]
            assert np.array_equal(got, ref_ms.c), f"position {pos} (pair {k})"
    ta, tb = c.lib.decrypt(c.s, ga), c.lib.decrypt(c.s, gb)
    got = c.lib.decrypt(c.s, prod)
    for pos in range(32):
        assert np.array_equal(got[pos], (ta[pos % 2].astype(object) * tb[pos % 2].astype(object)) % t)


def _noise_bits(c, ct):
    """log2 of the largest |c0 + c1 s| (centered mod q_0) over the coefficients of a level-1
    ciphertext: the plaintext (|m| <= t/2) plus t times the noise."""
    from oracle import _ring as R
    q0 = c.P.q[0]
    w = c.coeff_words(ct)[0]  # [2][level][N]
    s = np.mod(np.asarray(c.s, dtype=np.int64), q0).astype(np.uint64)
    phase = (w[0, 0].astype(object) + R.negacyclic_dot(w[1, 0], s, q0).astype(object)) % q0
    big = max(abs(int(v) - q0 if int(v) > q0 // 2 else int(v)) for v in phase)
    return math.log2(max(big, 1)), math.log2(q0 / 2)


def test_noise_margin_of_the_query_at_full_size():
    """The filter+SUM query at N = 2^16, L = 30, K = 6 with the dense ternary secret of the
    benchmark: its result decrypts to the plaintext query in both evaluation schedules, and the
    largest |c0 + c1 s| of the final ciphertext stays well below q_0 / 2, under the library's
    noise estimate.  The fast schedule lowers operands by dropping limbs where the estimate
    allows; the margin shows what that leaves."""
    log("[noise] N=2^16 L=30 K=6, dense ternary secret, 2 ciphertexts per column")
    c = Pair(16, 257, 2, 30, 6, steps=(1, 2, 4, 8, 16, 32), conj=True, oracle_keys=False)
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(77)
    cols = {k: g.integers(0, 1 << 16, size=(2, P.ell)) for k in "abc"}
    thr = int(g.integers(0, 1 << 16))
    A, Bc, C = (c.enc_both(cols[k], oracle=False)[0] for k in "abc")
    T = c.enc_both(np.full((1, P.ell), thr), oracle=False)[0]
    a, b, cc = (cols[k].astype(np.int64) for k in "abc")
    want = int((b * cc * (((a - thr) % t) > (t - 1) // 2)).sum() % t)
    margins = {}
    for sched in ("fast", "basic"):
        with schedule(c, sched):
            out = c.lib.filter_sum(c.keys, A, T, Bc, C)
        assert out.level >= 1
        assert all(int(v) == want for v in c.lib.decrypt(c.s, out)[0]), sched
        if out.level > 1:
            out = c.lib.mod_switch_to(out, 1)
        bits, half = _noise_bits(c, out)
        margins[sched] = half - bits
        log(f"[noise] {sched}: largest |c0 + c1 s| = 2^{bits:.1f} (estimate 2^{out.noise / 16:.1f}), "
            f"q_0 / 2 = 2^{half:.1f}")
        # the library's noise estimate bounds what was measured, and itself stays below q_0 / 2
        assert 0 < out.noise and bits <= out.noise / 16 < half, (sched, bits, out.noise / 16)
    assert min(margins.values()) >= 8, margins
