"""Host logic of the benchmark: the plaintext expectation of the filter query and its
agreement with the integer predicate (the comparison is on centered values of Z_{p^2},
so it equals a < t only when |a - t| <= (p^2 - 1)/2)."""
import numpy as np

import bench


def _cols(a, b=None, c=None):
    a = np.asarray(a, dtype=np.uint64).reshape(1, -1)
    ones = np.ones_like(a)
    return {"a": a, "b": ones if b is None else np.asarray(b, dtype=np.uint64).reshape(1, -1),
            "c": ones if c is None else np.asarray(c, dtype=np.uint64).reshape(1, -1)}


def test_expected_sum_counts_centered_negatives():
    t = 257 ** 2
    # a - thr = -1 (counted), 0, +1, and 65535 - 0 = 65535 > (t - 1)/2 (centered -514: counted)
    cols = _cols([9, 10, 11, 65535], b=[2, 3, 5, 7], c=[1, 1, 1, 11])
    assert bench.expected_sum(cols, 10) == (2 + 7 * 11) % t
    cols = _cols([65535], b=[7], c=[11])
    assert bench.expected_sum(cols, 0) == 77


def test_sql_agreement_edges():
    half = (257 ** 2 - 1) // 2  # 33024
    # |a - thr| = half agrees, half + 1 does not (a - thr = -(half + 1) is centered positive)
    ag = bench.sql_agreement(_cols([0, half + 1]), half + 1)
    assert ag["rows_agree"] == 0.5
    ag = bench.sql_agreement(_cols([1, half + 1]), half + 1)
    assert ag["rows_agree"] == 1.0 and ag["sum_equals_sql"]


def test_fifteen_bit_values_always_agree_and_sixteen_bit_do_not():
    g = np.random.default_rng(5)
    a15 = g.integers(0, 1 << 15, size=4096)
    for thr in (0, 1, 16384, (1 << 15) - 1):
        ag = bench.sql_agreement(_cols(a15), thr)
        assert ag["rows_agree"] == 1.0 and ag["sum_equals_sql"]
    # over all 16-bit (a, thr) pairs the disagreeing share is ((2^16 - 33025) / 2^16)^2 = 0.2461
    a16 = np.arange(1 << 16)
    bad = sum((1.0 - bench.sql_agreement(_cols(a16), int(thr))["rows_agree"]) for thr in range(0, 1 << 16, 64))
    share = bad / len(range(0, 1 << 16, 64))
    assert abs(share - ((65536 - 33025) / 65536) ** 2) < 2e-3


def test_cpu_baseline_schedule_replay_runs_and_restores_the_oracle():
    """The CPU baseline scales one oracle product by the limb products of the oracle's own
    schedule, replayed on level-only stand-ins; the replay must cover every oracle function the
    schedule calls and put them all back."""
    import oracle.bgv as OB
    before = {k: getattr(OB, k) for k in ("mul_relin", "mod_switch", "drop", "tensor", "relin", "align")}
    per_ct, tail = bench.limb_products_per_query_ct()
    assert per_ct > 0 and tail > 0
    assert all(getattr(OB, k) is v for k, v in before.items())
