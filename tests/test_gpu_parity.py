"""GPU parity: every library operation, called through the C-ABI, against the CPU oracle
on the same seeded inputs, word for word (tolerance 0: all arithmetic is exact integer)."""
import numpy as np
import pytest

from oracle import _ring as R
from oracle import bgv as B
from oracle import space as S
from oracle.params import Params
from tests.gpu_ctx import (Pair, log, pair_hybrid17, pair_r3_17, pair_r4_37, pair_tiny17, pair_tiny5, pair_tiny5_r3,
                           pair_tiny5_r4, schedule)

pytestmark = pytest.mark.gpu


def _rand_limbs(P, level, n_polys, seed):
    g = np.random.default_rng(seed)
    return np.stack([np.stack([g.integers(0, q, size=P.N, dtype=np.uint64) for q in P.primes[:level]])
                     for _ in range(n_polys)])


@pytest.mark.parametrize("logN", [4, 5, 8, 9, 10, 12])
def test_ntt_matches_the_definition(logN):
    import torch
    from paper_2604_19890_amd import bgv as G
    log(f"[ntt] logN={logN}")
    lib = G.Context(logN, 17, 2, 3, 1)
    P = Params(logN, 17, 2, 3, 1)
    x = _rand_limbs(P, 4, 2, logN)  # 2 polys x 4 limbs (3 q-primes + the special prime)
    t = torch.from_numpy(x.reshape(-1).view(np.int64).copy()).cuda()
    lib.ntt(t, 2, 4, inverse=False)
    got = t.cpu().numpy().view(np.uint64).reshape(x.shape)
    for b in range(2):
        for i, q in enumerate(P.primes[:4]):
            assert np.array_equal(got[b, i], R.ntt_def(x[b, i], q, P.psi(q))), (b, i)
    lib.ntt(t, 2, 4, inverse=True)
    assert np.array_equal(t.cpu().numpy().view(np.uint64).reshape(x.shape), x)


@pytest.mark.parametrize("logN,p", [(13, 17), (14, 257), (15, 257), (16, 257)])
def test_ntt_large_rings_sampled(logN, p):
    import torch
    from paper_2604_19890_amd import bgv as G
    log(f"[ntt-large] logN={logN}")
    lib = G.Context(logN, p, 2, 3, 2)
    P = Params(logN, p, 2, 3, 2)
    x = _rand_limbs(P, 5, 1, logN)
    t = torch.from_numpy(x.reshape(-1).view(np.int64).copy()).cuda()
    lib.ntt(t, 1, 5, inverse=False)
    got = t.cpu().numpy().view(np.uint64).reshape(x.shape)
    idx = np.array([0, 1, 2, 3, 777, P.N // 2 - 1, P.N // 2, P.N - 2, P.N - 1])
    for i, q in enumerate(P.primes[:5]):
        assert np.array_equal(got[0, i, idx], R.ntt_def_at(x[0, i], q, P.psi(q), idx)), i
    lib.ntt(t, 1, 5, inverse=True)
    assert np.array_equal(t.cpu().numpy().view(np.uint64).reshape(x.shape), x)


@pytest.mark.parametrize("pf", [pair_tiny5, pair_tiny17, pair_hybrid17])
def test_encrypt_and_decrypt_match(pf):
    c = pf()
    t = c.P.t_full
    rows = np.random.default_rng(1).integers(0, t, size=(3, c.P.ell))
    g, o = c.enc_both(rows)
    c.assert_equal(g, o, "encrypt")
    vals, flags = c.lib.decrypt(c.s, g, with_flags=True)
    assert np.array_equal(vals, rows) and not flags.any()
    for b in range(3):
        assert list(B.decrypt(c.P, c.s, o[b])[0]) == list(rows[b])


def test_linear_operations_match():
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(2)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    lib = c.lib
    c.assert_equal(lib.add(ga, gb), [B.add(P, x, y) for x, y in zip(oa, ob)], "add")
    c.assert_equal(lib.sub(ga, gb), [B.sub(P, x, y) for x, y in zip(oa, ob)], "sub")
    c.assert_equal(lib.negate(ga), [B.neg(P, x) for x in oa], "negate")
    c.assert_equal(lib.mul_scalar(ga, -12345), [B.mul_scalar(P, x, -12345) for x in oa], "mul_scalar")
    c.assert_equal(lib.add_const(ga, 200), [B.add_const(P, x, 200) for x in oa], "add_const")
    g1, o1 = c.enc_both(g.integers(0, t, size=(1, P.ell)))
    c.assert_equal(lib.add(ga, g1), [B.add(P, x, o1[0]) for x in oa], "broadcast add")
    gp, op_ = c.enc_both([[P.p * k for k in range(P.ell)]])
    c.assert_equal(lib.divide_by_p(gp), [B.divide_by_p(P, op_[0])], "divide_by_p")
    with pytest.raises(c.G.BgvError):
        lib.add(ga, lib.mod_switch(gb))


@pytest.mark.parametrize("pf", [pair_tiny5, pair_tiny17, pair_hybrid17])
def test_mul_relin_and_mod_switch_match(pf):
    c = pf()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(3)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    m = c.lib.mul_relin(c.keys, ga, gb)
    om = [B.mul_relin(P, c.okeys.relin, x, y) for x, y in zip(oa, ob)]
    c.assert_equal(m, om, "mul_relin")
    ms = c.lib.mod_switch(m)
    oms = [B.mod_switch(P, x) for x in om]
    c.assert_equal(ms, oms, "mod_switch")
    # in place: the output buffer is the input's
    m2 = c.lib.mul_relin(c.keys, ga, gb)
    c.assert_equal(c.lib.mod_switch(m2, out=m2), oms, "mod_switch in place")
    to = max(1, P.L - 4)
    mt = c.lib.mod_switch_to(m, to)
    c.assert_equal(mt, [B.align(P, x, to) for x in om], "mod_switch_to")
    # all the way down (more than 16 drops in chained launches where the chain is that long)
    c.assert_equal(c.lib.mod_switch_to(m, 1), [B.align(P, x, 1) for x in om], "mod_switch_to level 1")
    # in place, one step and chained
    for lv in (to, 1):
        m3 = c.lib.mul_relin(c.keys, ga, gb)
        c.assert_equal(c.lib.mod_switch_to(m3, lv, out=m3), [B.align(P, x, lv) for x in om],
                       f"mod_switch_to {lv} in place")
    # a product at a lower level (truncated last digit)
    la, lb = c.lib.mod_switch_to(ga, P.L - 3), c.lib.mod_switch_to(gb, P.L - 3)
    ol = [B.mul_relin(P, c.okeys.relin, B.align(P, x, P.L - 3), B.align(P, y, P.L - 3)) for x, y in zip(oa, ob)]
    c.assert_equal(c.lib.mul_relin(c.keys, la, lb), ol, "mul_relin low level")


@pytest.mark.parametrize("pf", [pair_tiny17, pair_hybrid17])
def test_rotate_matches(pf):
    c = pf()
    P, t = c.P, c.P.t_full
    ga, oa = c.enc_both(np.random.default_rng(4).integers(0, t, size=(2, P.ell)))
    for step in list(c.steps) + ([c.G.ROW_SWAP] if c.conj else []):
        ost = "conj" if step == c.G.ROW_SWAP else step
        c.assert_equal(c.lib.rotate(c.keys, ga, step), [B.rotate(P, c.okeys.galois, x, ost) for x in oa],
                       f"rotate {step}")


@pytest.mark.parametrize("sched", ["fast", "basic"])
@pytest.mark.parametrize("deg", [3, 16, 17, 30])
def test_eval_poly_matches(deg, sched):
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(deg)
    coeffs = [int(x) for x in g.integers(0, t, size=deg + 1)]
    coeffs[deg] = coeffs[deg] or 1
    if deg == 17:
        coeffs[0::2] = [0] * len(coeffs[0::2])  # an odd polynomial (sparse inner sums)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    with schedule(c, sched):
        out = c.lib.eval_poly(c.keys, ga, coeffs)
        c.assert_equal(out, [S.eval_poly(P, c.okeys, x, coeffs) for x in oa], f"eval_poly deg {deg} {sched}")


@pytest.mark.parametrize("pf,sched", [(pair_tiny5, "fast"), (pair_tiny17, "fast"), (pair_tiny5_r3, "fast"),
                                      (pair_r3_17, "fast"), (pair_tiny5_r4, "fast"), (pair_tiny5, "basic"),
                                      (pair_tiny17, "basic"), (pair_tiny5_r3, "basic")])
def test_space_switching_composites_match(pf, sched):
    with schedule(pf(), sched) as c:
        _composites(c)


def _composites(c):
    P, t = c.P, c.P.t_full
    rows = [[(i * 37 + b * 11) % t for i in range(P.ell)] for b in range(2)]
    ga, oa = c.enc_both(rows)
    gd = c.lib.space_reduce(c.keys, ga)
    od = [S.space_reduce(P, c.okeys, x) for x in oa]
    assert len(gd) == P.r
    for k in range(P.r):
        c.assert_equal(gd[k], [d[k] for d in od], f"reduce digit {k}")
    glt = c.lib.compare(c.keys, gd, c.G.OP_LT)
    olt = [S.compare(P, c.okeys, d, "lt") for d in od]
    c.assert_equal(glt, olt, "compare lt")
    geq = c.lib.compare(c.keys, gd, c.G.OP_EQ)
    c.assert_equal(geq, [S.compare(P, c.okeys, d, "eq") for d in od], "compare eq")
    for op, name in ((c.G.OP_GT, "gt"), (c.G.OP_LE, "le"), (c.G.OP_GE, "ge"), (c.G.OP_NEQ, "neq")):
        c.assert_equal(c.lib.compare(c.keys, gd, op), [S.compare(P, c.okeys, d, name) for d in od], f"compare {name}")
    graise = c.lib.space_raise(c.keys, glt)
    oraise = [S.space_raise(P, c.okeys, x) for x in olt]
    c.assert_equal(graise, oraise, "raise")
    expect = [[1 if (v % t) > (t - 1) // 2 else 0 for v in r] for r in rows]
    assert np.array_equal(c.lib.decrypt(c.s, graise), np.array(expect))


def test_reduce_compare_raise_table6_p37_r4():
    """p = 37, r = 4 (Table 6): the four digits, LT and its raise against the oracle."""
    c = pair_r4_37()
    P, t = c.P, c.P.t_full
    rows = [[0, t - 1], [(t - 1) // 2, (t + 1) // 2]]
    ga, oa = c.enc_both(rows)
    gd = c.lib.space_reduce(c.keys, ga)
    od = [S.space_reduce(P, c.okeys, x) for x in oa]
    assert len(gd) == 4
    for k in range(4):
        c.assert_equal(gd[k], [d[k] for d in od], f"reduce digit {k}")
    glt = c.lib.compare(c.keys, gd, c.G.OP_LT)
    olt = [S.compare(P, c.okeys, d, "lt") for d in od]
    c.assert_equal(glt, olt, "compare lt")
    graise = c.lib.space_raise(c.keys, glt)
    c.assert_equal(graise, [S.space_raise(P, c.okeys, x) for x in olt], "raise")
    assert np.array_equal(c.lib.decrypt(c.s, graise), np.array([[0, 1], [0, 1]]))


def test_rotate_sum_and_batch_equals_singles():
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    rows = np.random.default_rng(9).integers(0, t, size=(3, P.ell))
    ga, oa = c.enc_both(rows)
    rs = c.lib.rotate_sum(c.keys, ga)
    c.assert_equal(rs, [S.rotate_and_sum(P, c.okeys, x) for x in oa], "rotate_sum")
    assert np.array_equal(c.lib.decrypt(c.s, rs), np.array([[int(r.sum()) % t] * P.ell for r in rows]))
    # the batched call gives the same bits as one call per ciphertext
    m_batch = c.lib.mul_relin(c.keys, ga, ga)
    wb = c.coeff_words(m_batch)
    for b in range(3):
        single = c.lib.from_words(ga.words(P.N)[b:b + 1], ga.t_exp)
        single.level = ga.level
        ws = c.coeff_words(c.lib.mul_relin(c.keys, single, single))
        assert np.array_equal(ws[0], wb[b])


def test_workload_glue_matches():
    """bgv_mul, bgv_batch_sum, bgv_filter_sum and bgv_relu against the oracle's pipelines."""
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(12)
    a_rows = g.integers(0, t, size=(2, P.ell))
    b_rows = g.integers(0, 40, size=(2, P.ell))
    c_rows = g.integers(0, 40, size=(2, P.ell))
    ga, oa = c.enc_both(a_rows)
    gb, ob = c.enc_both(b_rows)
    gc, oc = c.enc_both(c_rows)
    gt, ot = c.enc_both([[100] * P.ell])
    m = c.lib.mul(c.keys, gb, gc)
    om = [S._mul(P, c.okeys, x, y) for x, y in zip(ob, oc)]
    c.assert_equal(m, om, "mul")
    gbc = c.lib.mul_scalar(gb, 1)  # a copy of gb's words
    c.assert_equal(c.lib.mul(c.keys, gbc, gc, out=gbc), om, "mul into its first operand")
    bs = c.lib.batch_sum(gb)
    c.assert_equal(bs, [B.add_many(P, ob)], "batch_sum")
    fs = c.lib.filter_sum(c.keys, ga, gt, gb, gc)
    prods = [S.filter_product(P, c.okeys, x, ot[0], y, z) for x, y, z in zip(oa, ob, oc)]
    ref = S.rotate_and_sum(P, c.okeys, B.add_many(P, prods))
    c.assert_equal(fs, [ref], "filter_sum")
    cen = lambda v: v - t if v > (t - 1) // 2 else v
    expect = sum(int(y) * int(z) for ra, rb, rc in zip(a_rows, b_rows, c_rows)
                 for x, y, z in zip(ra, rb, rc) if cen((int(x) - 100) % t) < 0) % t
    assert np.array_equal(c.lib.decrypt(c.s, fs), np.array([[expect] * P.ell]))
    r = c.lib.relu(c.keys, ga)
    c.assert_equal(r, [S.relu(P, c.okeys, x) for x in oa], "relu")



@pytest.mark.parametrize("logN", [10, 12, 14])
def test_every_ntt_split_matches_the_definition_and_autotune_picks_one(logN):
    import torch
    from paper_2604_19890_amd import bgv as G
    lib = G.Context(logN, 17, 2, 3, 1)
    P = Params(logN, 17, 2, 3, 1)
    x = _rand_limbs(P, 3, 1, logN + 100)
    idx = np.array([0, 1, 5, P.N // 2, P.N - 1])
    ref = [R.ntt_def_at(x[0, i], q, P.psi(q), idx) for i, q in enumerate(P.primes[:3])]
    for split in [s for s in range(4, 9) if 4 <= logN - s <= 8]:
        lib.set_ntt_split(split)
        t = torch.from_numpy(x.reshape(-1).view(np.int64).copy()).cuda()
        lib.ntt(t, 1, 3)
        got = t.cpu().numpy().view(np.uint64).reshape(x.shape)
        for i in range(3):
            assert np.array_equal(got[0, i, idx], ref[i]), (split, i)
        lib.ntt(t, 1, 3, inverse=True)
        assert np.array_equal(t.cpu().numpy().view(np.uint64).reshape(x.shape), x), split
    split, us = lib.autotune_ntt(64, reps=3)
    assert 4 <= split <= 8 and 4 <= logN - split <= 8 and us > 0
