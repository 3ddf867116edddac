"""Edge cases through the C-ABI: rejected arguments (typed statuses, decided on the host before
anything is enqueued), ragged and broadcast batches, and the degenerate cases of the method."""
import numpy as np
import pytest

from oracle import bgv as B
from oracle import space as S
from tests.gpu_ctx import pair_tiny17, pair_tiny5

pytestmark = pytest.mark.gpu


def _status(c, fn, *args, **kw):
    with pytest.raises(c.G.BgvError) as ei:
        fn(*args, **kw)
    return c.G.STATUS[ei.value.status]


def test_rejected_arguments_carry_their_status():
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(21)
    ga, _ = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    lib = c.lib
    # an empty batch
    empty = c.G.Ct(ga.tensor, 0, ga.level, ga.t_exp)
    assert _status(c, lib.negate, empty) == "E_ARG"
    # input and output buffers smaller than the batch they describe
    short_in = c.G.Ct(ga.tensor[: ga.tensor.numel() // 2], 2, ga.level, ga.t_exp)
    assert _status(c, lib.negate, short_in) == "E_ARG"
    short_out = lib.empty(1, ga.level)
    assert _status(c, lib.negate, ga, out=short_out) == "E_ARG"
    # a chain too short for the operation
    low = lib.mod_switch_to(ga, 1)
    assert _status(c, lib.mod_switch, low) == "E_LEVEL"
    assert _status(c, lib.mul, c.keys, low, low) == "E_LEVEL"
    assert _status(c, lib.eval_poly, c.keys, lib.mod_switch_to(ga, 2), [1, 2, 3, 4, 5, 6, 7, 8, 9]) == "E_LEVEL"
    # operands tagged with different plaintext moduli
    gp = lib.set_t_exp(lib.mul_scalar(ga, P.p), 1)
    assert _status(c, lib.add, ga, gp) == "E_PTXT_MOD"
    assert _status(c, lib.less_than, c.keys, gp, None) == "E_PTXT_MOD"
    # a rotation without its key (keys for steps 1 and 2 only)
    assert _status(c, lib.rotate, c.keys, ga, 3) == "E_NOKEY"
    # a constant polynomial has nothing to evaluate
    assert _status(c, lib.eval_poly, c.keys, ga, [5]) == "E_ARG"
    # the failed calls left the context usable
    assert np.array_equal(lib.decrypt(c.s, lib.add(ga, ga)), (2 * lib.decrypt(c.s, ga)) % t)


@pytest.mark.parametrize("n", [3, 5])
def test_ragged_batches_match(n):
    """Batch sizes that are not powers of two (products, switches, rotations)."""
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(30 + n)
    ga, oa = c.enc_both(g.integers(0, t, size=(n, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(n, P.ell)))
    c.assert_equal(c.lib.mul_relin(c.keys, ga, gb), [B.mul_relin(P, c.okeys.relin, x, y) for x, y in zip(oa, ob)],
                   f"mul_relin n={n}")
    c.assert_equal(c.lib.mod_switch_to(ga, P.L - 5), [B.align(P, x, P.L - 5) for x in oa], f"mod_switch_to n={n}")
    c.assert_equal(c.lib.rotate(c.keys, gb, 1), [B.rotate(P, c.okeys.galois, x, 1) for x in ob], f"rotate n={n}")


def test_broadcast_operand_matches():
    """One ciphertext against a batch of three (the encrypted threshold of the query)."""
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(40)
    ga, oa = c.enc_both(g.integers(0, t, size=(3, P.ell)))
    g1, o1 = c.enc_both(g.integers(0, t, size=(1, P.ell)))
    c.assert_equal(c.lib.sub(ga, g1), [B.sub(P, x, o1[0]) for x in oa], "sub broadcast")
    c.assert_equal(c.lib.mul(c.keys, ga, g1), [S._mul(P, c.okeys, x, o1[0]) for x in oa], "mul broadcast")


def test_degenerate_cases_match():
    """A linear polynomial (no product), the reduction of a value already in digit space (its
    single digit is the value itself), and comparison with one digit."""
    c = pair_tiny5()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(50)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    lin = c.lib.eval_poly(c.keys, ga, [3, 7])
    assert lin.level == ga.level
    c.assert_equal(lin, [S.eval_poly(P, c.okeys, x, [3, 7]) for x in oa], "linear polynomial")
    gp = c.lib.set_t_exp(ga, 1)
    digits = c.lib.space_reduce(c.keys, gp)
    assert len(digits) == 1
    op = [B.change_mod_to_p(P, x) for x in oa]
    c.assert_equal(digits[0], op, "reduce of a digit-space value")
    c.assert_equal(c.lib.compare(c.keys, digits, c.G.OP_LT), [S.compare(P, c.okeys, [x], "lt") for x in op],
                   "compare with one digit")


def test_batch_limit():
    """A call accepts up to max_batch ciphertexts (every launch of the call then fits the grid
    limits); one more is rejected before anything is enqueued."""
    c = pair_tiny17()
    P, t, lib = c.P, c.P.t_full, c.lib
    assert lib.max_batch == 65535 // (max(lib.dnum, 2) * (lib.L + lib.K))
    g = np.random.default_rng(60)
    m = g.integers(0, t, size=(1, P.ell))
    ga, _ = c.enc_both(m)
    full = lib.concat([ga] * lib.max_batch)
    got = lib.decrypt(c.s, lib.mul_scalar(full, 3))
    assert got.shape[0] == lib.max_batch
    assert np.array_equal(got[0], (3 * m[0]) % t) and np.array_equal(got[-1], (3 * m[0]) % t)
    over = lib.concat([full, ga])
    assert _status(c, lib.mul_scalar, over, 3) == "E_ARG"
    assert _status(c, lib.mod_switch, over) == "E_ARG"


def test_raw_ntt_and_autotune_limb_limit():
    """The raw transform and the split autotuner take at most 65535 limbs per call (the grid's y
    extent); beyond that they fail on the host with E_ARG instead of launching."""
    import torch
    c = pair_tiny17()
    lib = c.lib
    level = 5
    n_polys = 65535 // level + 1
    x = torch.zeros(n_polys * level * lib.N, dtype=torch.int64, device="cuda")
    assert _status(c, lib.ntt, x, n_polys, level) == "E_ARG"
    assert _status(c, lib.autotune_ntt, 65536, 1) == "E_ARG"
    lib.ntt(x, n_polys - 1, level)  # 65535 limbs: accepted (zeros stay zeros)
    torch.cuda.synchronize()
    assert int(x.abs().sum()) == 0


def test_unknown_schedule_is_rejected():
    c = pair_tiny17()
    assert c.G._lib.bgv_set_schedule(c.lib.handle, 7) == 1  # BGV_E_ARG
    with pytest.raises(KeyError):
        c.lib.set_schedule("fastest")
    c.lib.set_schedule("fast")


def test_fusion_settings_reject_unknown_modes():
    c = pair_tiny17()
    G, h = c.G._lib, c.lib.handle
    assert G.bgv_set_moddown_fused(h, 3) == 1 and G.bgv_set_moddown_fused(h, -1) == 1  # BGV_E_ARG
    assert G.bgv_set_modup_fused(h, 2) == 1
    for m in (0, 2, 1):
        assert G.bgv_set_moddown_fused(h, m) == 0


def test_noise_estimates_through_the_binding():
    """Every call that writes a batch gives it an estimate; a batch without one (noise 0) is
    lowered by rescaling switches only and still decrypts to the right values; concat keeps the
    largest estimate of its parts, or none if a part has none."""
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(41)
    ra, rb = g.integers(0, t, size=(2, P.ell)), g.integers(0, t, size=(2, P.ell))
    ga, _ = c.enc_both(ra, oracle=False)
    gb, _ = c.enc_both(rb, oracle=False)
    assert ga.noise > 0 and gb.noise == ga.noise
    c.lib.reset_stats()
    known = c.lib.less_than(c.keys, ga, gb)
    st_known = c.lib.stats()
    assert known.noise > 0
    c.lib.reset_stats()
    blind_a = c.G.Ct(ga.tensor, ga.n, ga.level, ga.t_exp)  # noise 0: unknown
    blind = c.lib.less_than(c.keys, blind_a, gb)
    st = c.lib.stats()
    assert blind.noise == 0 and st["rescale_drops"] > st_known["rescale_drops"]
    cen = lambda v: v - t if v > (t - 1) // 2 else v
    want = [[1 if cen((int(x) - int(y)) % t) < 0 else 0 for x, y in zip(r1, r2)] for r1, r2 in zip(ra, rb)]
    assert c.lib.decrypt(c.s, blind).tolist() == want
    assert c.lib.decrypt(c.s, known).tolist() == want
    both = c.lib.concat([ga, gb])
    assert both.noise == ga.noise
    assert c.lib.concat([ga, blind_a]).noise == 0


def test_batch_sum_of_many_matches_the_oracle():
    """bgv_batch_sum over batches of 1, 4 and 9 ciphertexts: the words and the noise estimate of
    the oracle's sum of n terms (a + ceil(16 log2 n); a chain of pairwise bounds would differ
    from four terms on), and the slot-wise sums under decryption."""
    from oracle import noise as NZ
    c = pair_tiny17()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(43)
    rows = g.integers(0, t, size=(9, P.ell))
    gx, ox = c.enc_both(rows)
    for n in (1, 4, 9):
        part = c.lib.view(gx, 0, n)
        s = c.lib.batch_sum(part)
        ref = B.add_many(P, ox[:n])
        c.assert_equal(s, [ref], f"batch_sum of {n}")
        assert s.noise == NZ.sum_of(ox[0].nz, n) == ref.nz
        assert c.lib.decrypt(c.s, s).tolist() == [[int(v) % t for v in rows[:n].sum(axis=0)]]
