"""The streamed whole-workload legs of the benchmark (bench.stream_query, bench.stream_relu)
on a small ring.

The full-size run (2^20 rows at N = 2^16) takes minutes, so the leg's bookkeeping is checked
here on the benchmark's plaintext modulus and chain at N = 2^10: several steps, a ragged
last step and a ragged last ciphertext.  The decrypted SUM must equal the plaintext SUM of
b * c over the rows whose circuit predicate holds."""
import pytest

import bench
from paper_2604_19890_amd import bgv as G
from paper_2604_19890_amd import synth
from tests.gpu_ctx import log

pytestmark = pytest.mark.gpu


def test_streamed_query_sums_every_row():
    log("[stream] N=2^10 p=257 r=2 L=30 K=6")
    ctx = G.Context(10, 257, 2, 30, 6)
    s = synth.ternary(ctx.N, 5, 3)
    keys = bench.make_keys(ctx, s, 3, 5, [1 << i for i in range(6)], True)
    rows = 5 * ctx.slots + 37  # three steps of two ciphertexts; the last holds 165 rows
    res = bench.stream_query(ctx, keys, s, rows, 2, seed=5, wl=3)
    assert res["rows"] == rows and res["steps"] == 3
    assert res["decrypted_sum_correct"], res
    assert 0.0 < res["rows_agree"] <= 1.0
    assert res["final_noise_bits"] > 0


def test_streamed_relu_is_right_on_every_activation():
    log("[stream] relu N=2^9 p=257 r=2 L=30 K=6")
    ctx = G.Context(9, 257, 2, 30, 6)
    s = synth.ternary(ctx.N, 7, 6)
    keys = bench.make_keys(ctx, s, 6, 7, [], False)
    total = 3 * ctx.slots + 50  # two calls of two ciphertexts; the last call is ragged
    res = bench.stream_relu(ctx, keys, s, total, 2, seed=7, wl=6)
    assert res["activations"] == total and res["calls"] == 2
    assert res["wrong"] == 0, res
