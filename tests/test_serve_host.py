"""Host logic of the served form (no GPU): which ring each query kind runs on, the chains the
rings keep, and the security estimate reported next to them."""


def test_ring_chains_hold_their_queries():
    """The serving rings' chains: arithmetic-only queries need one product and rotate-and-sum,
    the compare circuit 29 products; filter queries go to the ring that holds it."""
    from paper_2604_19890_amd import serve as SV
    assert SV.RING_CHAINS[14][0] >= 2 and SV.RING_CHAINS[15][0] >= 2 and SV.RING_CHAINS[16][0] >= 30
    qs = SV.make_queries(200, [14, 15, 16], 1 << 10, 1 << 12, rate=1.0)
    assert all(q.log_n == 16 for q in qs if q.kind == "filter")
    assert {q.log_n for q in qs if q.kind == "sum"} == {14, 15, 16}
    est = SV.security_estimate(16, 30, 6)
    assert est["log2_qp"] == 1800 and 120 <= est["lambda_est"] <= 128
