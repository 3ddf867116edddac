"""Served form: a query's result is the same alone and in a mix of queries, and equals the
plaintext query; admission by footprint rejects a query larger than the budget."""
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
