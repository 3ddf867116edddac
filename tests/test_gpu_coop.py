"""The XCD-local transform (one persistent launch per two-pass transform, intermediate kept in
L2) against the two-launch form, bit for bit: forward and inverse transforms over many limbs at
N = 2^14, 2^15 and 2^16 for several lookaheads, and the product step, rotation and repeated
modulus switching (out-of-place first passes, physical row maps, the epilogue pass) at the
benchmark's shape.

That form is switched off: the first GPU run of the first test below produced no output for
180 s and was stopped (no fault).  A CPU simulation of its work queue finds no deadlock at that
shape, and no defect of the code explaining the stall has been shown, so it is not run again;
the setter rejects it, and the equality tests are skipped with that reason."""
import numpy as np
import pytest

from paper_2604_19890_amd import synth

pytestmark = pytest.mark.gpu


def _rand(n_words, seed, q_max):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randint(0, q_max, (n_words,), dtype=torch.int64, generator=g).cuda()


SWITCHED_OFF = ("the XCD-local transform is switched off: its first GPU run stalled without output and "
                "no cause has been shown")


def test_the_xcd_local_form_is_rejected():
    from paper_2604_19890_amd import bgv as G
    ctx = G.Context(16, 257, 2, 3, 2)
    ctx.set_ntt_coop(0)
    with pytest.raises(G.BgvError) as ei:
        ctx.set_ntt_coop(1, 2)
    assert ei.value.status == 8  # BGV_E_UNSUPPORTED


@pytest.mark.skip(reason=SWITCHED_OFF)
@pytest.mark.parametrize("log_n,p,polys,level", [(14, 257, 24, 10), (15, 257, 12, 17), (16, 257, 32, 30)])
def test_xcd_local_transform_equals_two_launches(log_n, p, polys, level):
    from paper_2604_19890_amd import bgv as G
    ctx = G.Context(log_n, p, 2, max(level, 2), 2)
    qmin = min(ctx.primes[:level])
    x = _rand(polys * level * ctx.N, log_n, qmin)
    ctx.set_ntt_coop(0)
    ref_f = x.clone()
    ctx.ntt(ref_f, polys, level, inverse=False)
    ref_i = x.clone()
    ctx.ntt(ref_i, polys, level, inverse=True)
    for la in (0, 1, 2, 4):
        ctx.set_ntt_coop(1, la)
        y = x.clone()
        ctx.ntt(y, polys, level, inverse=False)
        z = x.clone()
        ctx.ntt(z, polys, level, inverse=True)
        ctx.sync()  # raises if a wait of the persistent form ran past its limit
        assert bool((y == ref_f).all()), f"forward, lookahead {la}"
        assert bool((z == ref_i).all()), f"inverse, lookahead {la}"
        ctx.ntt(y, polys, level, inverse=True)
        assert bool((y == x).all()), f"round trip, lookahead {la}"
    ctx.sync()


@pytest.mark.skip(reason=SWITCHED_OFF)
def test_xcd_local_form_in_the_product_step_rotation_and_switches():
    from paper_2604_19890_amd import bgv as G
    ctx = G.Context(16, 257, 2, 30, 6)
    N = ctx.N
    s = synth.ternary(N, 0, 94)
    n_keys = 2
    ka = np.empty((n_keys, ctx.dnum, ctx.L + ctx.K, N), dtype=np.uint64)
    ke = np.empty((n_keys, ctx.dnum, N), dtype=np.int32)
    for i in range(n_keys):
        ka[i], ke[i] = synth.key_randomness(ctx.primes, N, ctx.dnum, 0, 94, i)
    keys = ctx.keygen(s, ka, ke, steps=[1])
    g = np.random.default_rng(94)

    def enc(n, base):
        c1 = np.empty((n, ctx.L, N), dtype=np.uint64)
        e = np.empty((n, N), dtype=np.int32)
        for i in range(n):
            c1[i], e[i] = synth.encryption_randomness(ctx.primes[:ctx.L], N, 0, 94, base + i)
        return ctx.encrypt(s, g.integers(0, ctx.t, size=(n, ctx.slots), dtype=np.uint64), c1, e)

    a, b = enc(4, 0), enc(4, 10)
    outs = {}
    for mode in (0, 1):
        ctx.set_ntt_coop(mode)
        prod = ctx.mul(keys, a, b)
        rot = ctx.rotate(keys, a, 1)
        sw = ctx.mod_switch_to(b, 7)
        rl = ctx.mul_relin(keys, a, b)
        ctx.sync()
        outs[mode] = [t.words(N) for t in (prod, rot, sw, rl)]
    for name, w0, w1 in zip(("product step", "rotate", "mod_switch_to", "mul_relin"), outs[0], outs[1]):
        assert np.array_equal(w0, w1), name
    # and the result still decrypts to the slot products
    ta, tb = ctx.decrypt(s, a), ctx.decrypt(s, b)
    got = ctx.decrypt(s, ctx.mul(keys, a, b))
    assert np.array_equal(got, (ta.astype(object) * tb.astype(object)) % ctx.t)
