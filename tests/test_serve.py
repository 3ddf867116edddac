"""Served form: each query's result ciphertext equals the oracle's pipeline on the same inputs
word for word, is the same alone and in a mix of queries, and decrypts to the plaintext query;
admission by footprint rejects a query larger than the budget."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _engine():
    from paper_2604_19890_amd import serve as SV
    return SV, {8: SV.Engine(8, 30, 6)}


def test_alone_and_in_the_mix_are_identical():
    SV, engines = _engine()
    qs = [SV.Query(i, 8, kind, rows, 0.0) for i, (kind, rows) in enumerate([("filter", 300), ("sum", 128), ("filter", 700)])]
    SV.prepare(qs, engines)
    alone = []
    for q in qs:
        SV.serve([q], engines, mode="batched", round_cts={8: 2})
        alone.append(q.result.tensor[: engines[8].ctx.words(q.result.level)].clone())
    stats = SV.serve(qs, engines, mode="batched", round_cts={8: 4})
    assert stats["queries"] == 3
    for q, ref in zip(qs, alone):
        got = q.result.tensor[: engines[8].ctx.words(q.result.level)]
        assert torch_equal(got, ref), f"query {q.qid} differs alone vs in the mix"
    assert SV.check(qs, engines) == 0
    plain = SV.serve(qs, engines, mode="plain")
    assert plain["queries"] == 3
    for q, ref in zip(qs, alone):
        assert torch_equal(q.result.tensor[: engines[8].ctx.words(q.result.level)], ref)


def test_served_results_match_the_oracle():
    """Per query: [a < t] * (b * c) (filter) or b * c (sum) per ciphertext, summed over the
    query's ciphertexts, then rotate-and-sum -- the oracle on the same keys and encryption
    randomness, against the served result; rounds of three ciphertexts split the queries across
    batches and mix them."""
    from oracle import bgv as B
    from oracle import space as S
    from oracle.params import Params
    from paper_2604_19890_amd import synth
    SV, engines = _engine()
    e = engines[8]
    qs = [SV.Query(i, 8, kind, rows, 0.0) for i, (kind, rows) in enumerate([("filter", 250), ("sum", 128), ("filter", 130)])]
    SV.prepare(qs, engines)
    SV.serve(qs, engines, mode="batched", round_cts={8: 3})
    P = Params(8, SV.P_, SV.R_, 30, 6)
    assert P.primes == e.ctx.primes
    kr = [synth.key_randomness(P.primes, P.N, P.dnum, 0, e.wl, i) for i in range(2 + len(SV.STEPS))]
    okeys = B.keygen(P, e.s, kr, steps=SV.STEPS, with_conj=True)

    def oenc(rows, base):
        out = []
        for i, r in enumerate(rows):
            c1, er = synth.encryption_randomness(P.q, P.N, 0, e.wl, base + i)
            out.append(B.encrypt(P, e.s, [int(v) for v in r], c1, er))
        return out

    for q in qs:
        base = 1000000 * (q.qid + 1)
        ob, oc = oenc(q.cols["b"], base + 300000), oenc(q.cols["c"], base + 600000)
        if q.kind == "filter":
            oa = oenc(q.cols["a"], base)
            ot = oenc([[q.thr] * P.ell], base + 900000)[0]
            prods = [S.filter_product(P, okeys, x, ot, y, z) for x, y, z in zip(oa, ob, oc)]
        else:
            prods = [S._mul(P, okeys, y, z) for y, z in zip(ob, oc)]
        ref = S.rotate_and_sum(P, okeys, B.add_many(P, prods))
        r = q.result
        w = r.tensor[: e.ctx.words(r.level)].clone()
        e.ctx.ntt(w, 2, r.level, inverse=True)
        got = w.cpu().numpy().view(np.uint64).reshape(2, r.level, P.N)
        assert (r.level, r.t_exp) == (ref.level, ref.t_exp), q.qid
        assert np.array_equal(got, ref.c), f"query {q.qid} ({q.kind}, {q.n_cts} ciphertexts)"
    assert SV.check(qs, engines) == 0


def test_admission_rejects_an_oversized_query():
    SV, engines = _engine()
    qs = [SV.Query(0, 8, "sum", 200, 0.0), SV.Query(1, 8, "sum", 100, 0.0)]
    SV.prepare(qs, engines)
    key_bytes = engines[8].keys.bytes
    budget = key_bytes + qs[1].footprint + 1  # fits the small query only
    stats = SV.serve(qs, engines, mode="batched", round_cts={8: 4}, budget_bytes=budget)
    assert stats["rejected"] == 1 and stats["queries"] == 1
    assert SV.check([qs[1]], engines) == 0


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))
