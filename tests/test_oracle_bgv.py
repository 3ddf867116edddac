"""Pins for the oracle's BGV operations: definitions, invariants and brute force."""
import numpy as np
import pytest

from oracle import bgv as B
from oracle import _ring as R
from oracle.params import Params
from tests.oracle_ctx import tiny5, tiny17, hybrid17


def _crt(residues, primes):
    Q = 1
    for q in primes:
        Q *= q
    x = 0
    for v, q in zip(residues, primes):
        Qh = Q // q
        x += int(v) * Qh * pow(Qh % q, -1, q)
    x %= Q
    return x - Q if x > Q // 2 else x, Q


@pytest.mark.parametrize("args", [(4, 5, 2), (5, 17, 2), (8, 257, 2)])
def test_encode_interpolates_the_slot_values(args):
    P = Params(*args, 2, 1)
    t = P.t_full
    g = np.random.default_rng(7)
    v = g.integers(0, t, size=P.ell)
    m = B.encode(P, v, P.r)
    assert all(m[i] == 0 for i in range(P.N) if i % P.d)
    assert all(-(t - 1) // 2 <= int(x) <= (t - 1) // 2 for x in m)
    # definition: M(zeta_j) = v_j with M(Y) = sum_k m_{kd} Y^k
    for j, z in enumerate(P.slot_roots(P.r)):
        assert sum(int(m[k * P.d]) * pow(z, k, t) for k in range(P.ell)) % t == v[j]
    vals, nonconst = B.decode(P, [int(x) % t for x in m], P.r)
    assert list(vals) == list(v) and not nonconst.any()
    # the all-c slot vector is the constant polynomial c
    mc = B.encode(P, [3] * P.ell, P.r)
    assert mc[0] == 3 and not mc[1:].any()


def test_decode_flags_nonconstant_slots():
    P = Params(5, 17, 2, 2, 1)
    m = [0] * P.N
    m[1] = 1  # X lies in no Z_{p^r} constant slot
    _, nonconst = B.decode(P, m, P.r)
    assert nonconst.all()


@pytest.mark.parametrize("ctx", [tiny5, tiny17])
def test_encrypt_decrypt_and_fresh_noise(ctx):
    c = ctx()
    P = c.P
    v = list(np.random.default_rng(1).integers(0, P.t_full, size=P.ell))
    ct = c.enc(v)
    vals, nonconst, bits = B.decrypt(P, c.s, ct)
    assert list(vals) == v and not nonconst.any()
    # fresh phase = m + t e: |m| <= (t-1)/2 and |e| <= 19
    assert bits <= (P.t_full * 19 + P.t_full).bit_length()


def test_linear_operations_act_slotwise():
    c = tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(2)
    a, b = [list(g.integers(0, t, size=P.ell)) for _ in range(2)]
    A, Bc = c.enc(a), c.enc(b)
    assert c.dec(B.add(P, A, Bc)) == [(x + y) % t for x, y in zip(a, b)]
    assert c.dec(B.sub(P, A, Bc)) == [(x - y) % t for x, y in zip(a, b)]
    assert c.dec(B.neg(P, A)) == [(-x) % t for x in a]
    assert c.dec(B.mul_scalar(P, A, 200)) == [(200 * x) % t for x in a]
    assert c.dec(B.add_const(P, A, 250)) == [(250 + x) % t for x in a]
    with pytest.raises(ValueError):
        B.add(P, A, B.mod_switch(P, Bc))


def test_sum_of_many_is_the_chained_sum():
    """add_many: the same words as pairwise additions, slot-wise sums under decryption, and
    level checks; only its estimate differs (n terms bounded by the largest)."""
    c = tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(21)
    rows = [list(g.integers(0, t, size=P.ell)) for _ in range(6)]
    cts = [c.enc(r) for r in rows]
    tot = B.add_many(P, cts)
    chain = cts[0]
    for x in cts[1:]:
        chain = B.add(P, chain, x)
    assert np.array_equal(tot.c, chain.c) and (tot.level, tot.t_exp) == (chain.level, chain.t_exp)
    assert c.dec(tot) == [sum(col) % t for col in zip(*rows)]
    assert B.add_many(P, cts[:1]).nz == cts[0].nz and np.array_equal(B.add_many(P, cts[:1]).c, cts[0].c)
    assert tot.nz < chain.nz
    with pytest.raises(ValueError):
        B.add_many(P, [cts[0], B.mod_switch(P, cts[1])])


@pytest.mark.parametrize("ctx", [tiny5, tiny17])
def test_mod_switch_is_the_nearest_congruent_rescaling(ctx):
    """BGV modulus switching: the output (as an integer mod Q') is the integer x closest to
    C / q_top with x = C (mod t), found here by brute force over bigints."""
    c = ctx()
    P = c.P
    ct = c.enc(list(range(P.ell)))
    ct = B.mul_relin(P, c.keys.relin, ct, ct)  # large phase noise, nontrivial w
    out = B.mod_switch(P, ct)
    t = P.t(ct.t_exp)
    qtop = P.q[ct.level - 1]
    for k in range(2):
        for n in (0, 1, P.N // 2, P.N - 1):
            C, Q = _crt(ct.c[k, :, n], P.q[: ct.level])
            got, Qp = _crt(out.c[k, :, n], P.q[: out.level])
            base = C // qtop
            best = min((x for x in range(base - 2 * t, base + 2 * t + 1) if (x - C) % t == 0),
                       key=lambda x: abs(x * qtop - C))
            assert (got - best) % Qp == 0
    assert c.dec(out) == c.dec(ct)


@pytest.mark.parametrize("ctx", [tiny17, hybrid17])
def test_mod_down_matches_its_integer_definition(ctx):
    """ModDown output o satisfies o * P = U - delta over the integers (mod Q), with
    delta = t * sum_k [w_k Phat_k^-1]_{p_k} Phat_k, w_k = [U t^-1]_{p_k}."""
    c = ctx()
    P = c.P
    lv = P.L - 1
    g = np.random.default_rng(3)
    u = np.stack([g.integers(0, q, size=P.N, dtype=np.uint64) for q in P.q[:lv] + P.P])
    t = P.t_full
    o = B.mod_down(P, u, lv, t)
    primes = P.q[:lv] + P.P
    Pp = 1
    for pk in P.P:
        Pp *= pk
    for n in (0, 3, P.N - 1):
        U, QP = _crt(u[:, n], primes)
        delta = 0
        for k, pk in enumerate(P.P):
            wk = int(u[lv + k, n]) * pow(t, -1, pk) % pk
            ph = Pp // pk
            delta += wk * pow(ph % pk, -1, pk) % pk * ph
        delta *= t
        assert (U - delta) % Pp == 0
        assert delta % t == 0 and (delta - U) % Pp == 0
        o_int, Q = _crt(o[:, n], P.q[:lv])
        assert (o_int * Pp - (U - delta)) % Q == 0


@pytest.mark.parametrize("ctx", [tiny5, tiny17, hybrid17])
def test_relinearised_product_decrypts_to_the_slot_product(ctx):
    c = ctx()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(4)
    a, b = [list(g.integers(0, t, size=P.ell)) for _ in range(2)]
    A, Bc = c.enc(a), c.enc(b)
    prod = B.mul_relin(P, c.keys.relin, A, Bc)
    assert c.dec(prod) == [x * y % t for x, y in zip(a, b)]
    # key switching adds little noise: the product of two fresh phases dominates
    _, _, bits = B.decrypt(P, c.s, prod)
    assert bits <= 2 * (P.t_full * 20).bit_length() + P.logN + 2
    # at a lower level too (truncated last digit)
    A2, B2 = B.align(P, A, P.L - 3), B.align(P, Bc, P.L - 3)
    assert c.dec(B.mul_relin(P, c.keys.relin, A2, B2)) == [x * y % t for x, y in zip(a, b)]


@pytest.mark.parametrize("ctx", [tiny17, hybrid17])
def test_rotation_permutes_slots_as_the_galois_action(ctx):
    c = ctx()
    P, t = c.P, c.P.t_full
    v = list(range(1, P.ell + 1))
    ct = c.enc(v)
    roots = P.slot_roots(P.r)
    for step in (1, "conj"):
        g = B.galois_elt(P, step)
        # new slot j holds old slot j' with zeta_{j'} = zeta_j^g
        expect = [v[roots.index(pow(z, g, t))] for z in roots]
        assert c.dec(B.rotate(P, c.keys.galois, ct, step)) == expect
        if step == 1:
            half = P.ell // 2
            assert expect == [v[(j + 1) % half + (j // half) * half] for j in range(P.ell)]


def test_divide_by_p_and_tag_changes():
    c = tiny17()
    P = c.P
    p = P.p
    v = [p * k for k in range(P.ell)]
    ct = c.enc(v)
    d = B.divide_by_p(P, ct)
    assert d.t_exp == 1 and c.dec(d) == [k % p for k in range(P.ell)]
    w = c.enc([20, 35, 1, 2, 3, 4, 5, 6])
    assert c.dec(B.change_mod_to_p(P, w)) == [x % p for x in [20, 35, 1, 2, 3, 4, 5, 6]]


def test_depth_example_ab_cd():
    """(ab)(cd): three multiplications, depth two (Background, BGV subsection)."""
    import os
    gold = dict(ln.split() for ln in open(os.path.join(os.path.dirname(__file__), "golden", "depth_example.txt"))
                if not ln.startswith("#"))
    from oracle import space as S
    c = tiny17()
    P, t = c.P, c.P.t_full
    a, b, cc, d = (c.enc([x] * P.ell) for x in (3, 5, 7, 11))
    cnt = S.Counter()
    ab = S._mul(P, c.keys, a, b, cnt)
    cd = S._mul(P, c.keys, cc, d, cnt)
    r = S._mul(P, c.keys, ab, cd, cnt)
    assert cnt.mul == int(gold["multiplications"])
    assert P.L - r.level == int(gold["depth"])
    assert c.dec(r) == [3 * 5 * 7 * 11 % t] * P.ell


@pytest.mark.parametrize("ctx", [tiny17, hybrid17])
def test_sampled_oracle_matches_full_oracle(ctx):
    """The sampled-output forms used at large rings agree with the full computations."""
    from paper_2604_19890_amd import synth
    c = ctx()
    P = c.P
    a, b = c.enc(list(range(P.ell))), c.enc([3] * P.ell)
    idx = [0, 5, P.N - 1]
    assert np.array_equal(B.mul_relin(P, c.keys.relin, a, b).c[:, :, idx], B.mul_relin_at(P, c.keys.relin, a, b, idx))
    assert np.array_equal(B.rotate(P, c.keys.galois, a, 1).c[:, :, idx], B.rotate_at(P, c.keys.galois, a, 1, idx))
    c1, e = synth.encryption_randomness(P.q, P.N, 0, 5, 3)
    ct = B.encrypt(P, c.s, list(range(P.ell)), c1, e)
    assert np.array_equal(ct.c[0][:, idx], B.encrypt_at(P, c.s, list(range(P.ell)), c1, e, idx))
