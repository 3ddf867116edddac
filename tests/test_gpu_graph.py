"""hipGraph capture of library operations: every replay gives the eager result, with eager
work and synchronisations between the replays, and the eager result is the oracle's, word for
word."""
import numpy as np
import pytest

from oracle import space as S
from tests.gpu_ctx import pair_two_pass_deep

pytestmark = pytest.mark.gpu


def test_captured_pipeline_replays_bit_exactly():
    import torch
    c = pair_two_pass_deep()
    P, t = c.P, c.P.t_full
    g = np.random.default_rng(31)
    ga, oa = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    gb, ob = c.enc_both(g.integers(0, t, size=(2, P.ell)))
    lib = c.lib
    out_lt = lib.empty(2, P.L)
    out_m = lib.empty(2, P.L)
    # eager reference (also builds the tables the capture will use)
    lib.less_than(c.keys, ga, gb, out=out_lt)
    lib.mul(c.keys, out_lt, ga, out=out_m)
    torch.cuda.synchronize()
    # the eager results against the oracle's pipeline on the same inputs
    o_lt = [S.less_than(P, c.okeys, x, y) for x, y in zip(oa, ob)]
    c.assert_equal(out_lt, o_lt, "less_than")
    c.assert_equal(out_m, [S._mul(P, c.okeys, l, x) for l, x in zip(o_lt, oa)], "masked product")
    # the words a result occupies (the buffers are sized for the top level; the rest is not written)
    w_lt, w_m = out_lt.n * lib.words(out_lt.level), out_m.n * lib.words(out_m.level)
    ref_lt = out_lt.tensor[:w_lt].clone()
    ref_m = out_m.tensor[:w_m].clone()
    ref_level = out_m.level
    out_lt.tensor.zero_()
    out_m.tensor.zero_()
    torch.cuda.synchronize()
    lib.capture_begin()
    lib.less_than(c.keys, ga, gb, out=out_lt)
    lib.mul(c.keys, out_lt, ga, out=out_m)
    graph = lib.capture_end()
    for rep in range(3):
        out_lt.tensor.zero_()
        out_m.tensor.zero_()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(out_lt.tensor[:w_lt], ref_lt), f"replay {rep}: less_than differs"
        assert torch.equal(out_m.tensor[:w_m], ref_m), f"replay {rep}: product differs"
        # eager work between replays
        lib.mul(c.keys, gb, gb)
        torch.cuda.synchronize()
    out_m.level = ref_level
    def lt(x, y):  # [centered(x - y) < 0] on Z_t
        return (int(x) - int(y)) % t > (t - 1) // 2
    expect = [[(int(v) if lt(x, y) else 0) for v, x, y in zip(av, av, bv)]
              for av, bv in zip(lib.decrypt(c.s, ga), lib.decrypt(c.s, gb))]
    assert np.array_equal(lib.decrypt(c.s, out_m), np.array(expect) % t)
    del graph
