"""Served form: continuous batching of encrypted filter-and-aggregate queries.

Queries arrive over time (Poisson arrivals), each with its own ring size, row count and
kind: SUM(b*c WHERE a < t) ("filter") or SUM(b*c) ("sum").  Rings keep the chains of the
serving configuration: 8 primes at N = 2^14 and 16 at N = 2^15 (special primes K = L / 4),
which hold the arithmetic-only query (one product, then rotate-and-sum).  The compare
circuit is 29 products deep, so filter queries run on the N = 2^16 ring, whose chain is
30 + 6 primes (the configured 24 extended to the circuit's depth).  Their encrypted columns are
resident in HBM; every ring keeps its evaluation keys resident.  A query is admitted when
its ciphertext footprint fits the memory budget next to the resident keys, and waits (FIFO)
otherwise; a query larger than the whole budget is rejected.

Batched mode: per ring, a scheduling round takes ciphertext chunks from the ring's queue,
the queries with the fewest ciphertexts left first (ties by arrival; policy "srpt", the
default) or in admission order (policy "fifo") -- several queries,
large queries split across rounds -- concatenates them into
one batch and runs the per-ciphertext products in one set of launches on the ring's stream
(rings run on separate streams, so their rounds overlap on the device).  Each query's products
are summed over its own ciphertexts and added to its running total; when the last chunk is
done the total goes through rotate-and-sum and the query completes.  Requests that arrive
while a round is on the GPU join the next round.

Plain mode: queries are served one at a time in arrival order, one ciphertext per call.

Latency = arrival to result ciphertext ready (device events against a common start event).
Every product is independent per ciphertext and the sums are exact modular additions, so a
query's result is the same alone and in any mix.
"""
from __future__ import annotations

import dataclasses
import json
import math
import time

import numpy as np
import torch

from . import bgv as G
from . import synth

P_, R_ = 257, 2
STEPS = [1 << i for i in range(6)]
# (ciphertext primes L, special primes K) per ring (log2 N)
RING_CHAINS = {14: (8, 2), 15: (16, 4), 16: (30, 6)}
# log2(Q P) bound for 128-bit security with a uniform ternary secret, from the homomorphic
# encryption security standard's table (N = 2^14, 2^15, 2^16)
QP_BITS_128 = {14: 438, 15: 881, 16: 1772}


def security_estimate(log_n: int, L: int, K: int, bits: int = 50) -> dict:
    """log2(Q P) of a chain and a rough security level: 128 scaled by the standard's log2(Q P)
    bound over the chain's (the level falls about in proportion to log2(Q P) at fixed N).
    An estimate for orientation, not the output of a lattice estimator."""
    qp = (L + K) * bits
    bound = QP_BITS_128.get(log_n)
    return {"log2_qp": qp, "bound_128": bound, "lambda_est": None if bound is None else round(128.0 * bound / qp)}


@dataclasses.dataclass
class Query:
    qid: int
    log_n: int
    kind: str
    rows: int
    arrival: float
    cols: dict = None  # plaintext columns (uint64 [n_cts][128]) and threshold, for checking
    thr: int = 0
    a: object = None
    b: object = None
    c: object = None
    t: object = None
    n_cts: int = 0
    next_ct: int = 0
    done_cts: int = 0
    partial: object = None
    result: object = None
    done_event: object = None
    latency_ms: float = None
    footprint: int = 0


class Engine:
    """One ring: context, resident keys, stream."""

    def __init__(self, log_n: int, L: int, K: int, seed: int = 0):
        self.log_n = log_n
        self.stream = torch.cuda.Stream()  # default priority
        with torch.cuda.stream(self.stream):
            self.ctx = G.Context(log_n, P_, R_, L, K, stream=self.stream)
            N = self.ctx.N
            wl = 40 + log_n
            self.s = synth.ternary(N, seed, wl)
            n_keys = 1 + len(STEPS) + 1
            ka = np.empty((n_keys, self.ctx.dnum, self.ctx.L + self.ctx.K, N), dtype=np.uint64)
            ke = np.empty((n_keys, self.ctx.dnum, N), dtype=np.int32)
            for i in range(n_keys):
                ka[i], ke[i] = synth.key_randomness(self.ctx.primes, N, self.ctx.dnum, seed, wl, i)
            self.keys = self.ctx.keygen(self.s, ka, ke, steps=STEPS, with_conj=True)
        self.wl = 40 + log_n
        self.ct_bytes = self.ctx.words(self.ctx.L) * 8
        # NTT pass split for this ring, picked by the autotuner on a round's transform shape
        with torch.cuda.stream(self.stream):
            self.ntt_split, self.ntt_split_us = self.ctx.autotune_ntt(
                min(32 << (16 - log_n), self.ctx.max_batch) * 2 * self.ctx.L, reps=3)
        self.busy = None  # (segments, event) of the round on the GPU
        self.queue = []

    def encrypt(self, rows: np.ndarray, index: int, seed: int = 0):
        ctx = self.ctx
        c1 = np.empty((len(rows), ctx.L, ctx.N), dtype=np.uint64)
        e = np.empty((len(rows), ctx.N), dtype=np.int32)
        for i in range(len(rows)):
            c1[i], e[i] = synth.encryption_randomness(ctx.primes[:ctx.L], ctx.N, seed, self.wl, index + i)
        with torch.cuda.stream(self.stream):
            return ctx.encrypt(self.s, rows, c1, e)

    # ------------------------------------------------------------------ batched rounds
    def launch_round(self, segments):
        """segments: list of (query, start, count).  Enqueue the round on the ring's stream."""
        ctx, keys = self.ctx, self.keys
        with torch.cuda.stream(self.stream):
            for kind in ("filter", "sum"):
                seg = [s for s in segments if s[0].kind == kind]
                if not seg:
                    continue
                B = ctx.concat([ctx.view(q.b, st, n) for q, st, n in seg])
                C = ctx.concat([ctx.view(q.c, st, n) for q, st, n in seg])
                if kind == "filter":
                    A = ctx.concat([ctx.view(q.a, st, n) for q, st, n in seg])
                    T = ctx.concat([q.t for q, st, n in seg for _ in range(n)])
                    prods = ctx.filter_products(keys, A, T, B, C)
                else:
                    prods = ctx.mul(keys, B, C)
                off = 0
                for q, st, n in seg:
                    part = ctx.batch_sum(ctx.view(prods, off, n))
                    q.partial = part if q.partial is None else ctx.add(q.partial, part)
                    off += n
            for q, st, n in segments:
                q.done_cts += n
                if q.done_cts == q.n_cts:
                    q.result = ctx.rotate_sum(keys, q.partial)
                    q.done_event = torch.cuda.Event(enable_timing=True)
                    q.done_event.record(self.stream)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.busy = (segments, ev)

    def run_plain(self, q: Query):
        """One ciphertext per call."""
        ctx, keys = self.ctx, self.keys
        with torch.cuda.stream(self.stream):
            for i in range(q.n_cts):
                b, c = ctx.view(q.b, i, 1), ctx.view(q.c, i, 1)
                if q.kind == "filter":
                    prod = ctx.filter_products(keys, ctx.view(q.a, i, 1), q.t, b, c)
                else:
                    prod = ctx.mul(keys, b, c)
                q.partial = prod if q.partial is None else ctx.add(q.partial, prod)
            q.result = ctx.rotate_sum(keys, q.partial)
            q.done_event = torch.cuda.Event(enable_timing=True)
            q.done_event.record(self.stream)


def make_queries(n_queries: int, rings, rows_lo: int, rows_hi: int, rate: float, seed: int = 0,
                 filter_ring: int = 16):
    """70% filter / 30% arithmetic-only queries, rows log-uniform in [rows_lo, rows_hi]; an
    arithmetic-only query takes a ring drawn uniformly from `rings`, a filter query the ring
    whose chain holds the compare circuit (filter_ring)."""
    g = synth.rng(seed, 77, synth.SLOTS, 0)
    t = 0.0
    out = []
    for i in range(n_queries):
        t += g.exponential(1.0 / rate) if rate > 0 else 0.0
        rows = int(round(math.exp(g.uniform(math.log(rows_lo), math.log(rows_hi)))))
        log_n = int(g.choice(rings))
        kind = "filter" if g.uniform() < 0.7 else "sum"
        if kind == "filter":
            log_n = filter_ring
        out.append(Query(i, log_n, kind, rows, t))
    return out


def prepare(queries, engines, seed: int = 0):
    """Encrypt every query's columns (client side, before serving starts)."""
    for q in queries:
        e = engines[q.log_n]
        ell = e.ctx.slots
        q.n_cts = -(-q.rows // ell)
        g = synth.rng(seed, 78, synth.SLOTS, q.qid)
        cols = {}
        for k in "abc":
            v = g.integers(0, 1 << 16, size=q.n_cts * ell, dtype=np.uint64)
            v[q.rows:] = 0  # padding rows contribute b*c = 0
            cols[k] = v.reshape(q.n_cts, ell)
        q.thr = int(g.integers(0, 1 << 16))
        q.cols = cols
        base = 1000000 * (q.qid + 1)
        q.a = e.encrypt(cols["a"], base) if q.kind == "filter" else None
        q.b = e.encrypt(cols["b"], base + 300000)
        q.c = e.encrypt(cols["c"], base + 600000)
        q.t = e.encrypt(np.full((1, ell), q.thr, dtype=np.uint64), base + 900000) if q.kind == "filter" else None
        q.footprint = (3 if q.kind == "filter" else 2) * q.n_cts * e.ct_bytes
    torch.cuda.synchronize()


def expected(q: Query, t=P_ ** R_) -> int:
    a, b, c = (q.cols[k].astype(np.int64) for k in "abc")
    if q.kind == "sum":
        return int((b * c).sum() % t)
    d = (a - q.thr) % t
    return int((b * c * (d > (t - 1) // 2)).sum() % t)


def release_cache(engines):
    for e in engines.values():
        e.ctx.trim()
    torch.cuda.empty_cache()


def reset(queries):
    for q in queries:
        q.next_ct = q.done_cts = 0
        q.partial = q.result = q.done_event = None
        q.latency_ms = None


def serve(queries, engines, mode: str = "batched", round_cts: dict = None, budget_bytes: float = 200e9,
          policy: str = "srpt"):
    """Serve the queries in real time; returns stats.  round_cts[log_n] bounds a round's batch."""
    reset(queries)
    key_bytes = sum(e.keys.bytes for e in engines.values())
    pending = sorted(queries, key=lambda q: q.arrival)
    rejected = [q for q in pending if q.footprint + key_bytes > budget_bytes]
    pending = [q for q in pending if q not in rejected]
    torch.cuda.synchronize()
    start_ev = torch.cuda.Event(enable_timing=True)
    start_ev.record()
    t0 = time.perf_counter()
    admitted, in_use = [], key_bytes
    waiting = list(pending)
    done = []
    while len(done) < len(pending):
        now = time.perf_counter() - t0
        # admission by footprint, FIFO
        while waiting and waiting[0].arrival <= now and in_use + waiting[0].footprint <= budget_bytes:
            q = waiting.pop(0)
            in_use += q.footprint
            admitted.append(q)
            engines[q.log_n].queue.append(q)
        if mode == "plain":
            if admitted:
                q = admitted.pop(0)
                engines[q.log_n].queue.remove(q)
                engines[q.log_n].run_plain(q)
                q.done_event.synchronize()
                done.append(q)
                in_use -= q.footprint
            elif waiting:
                time.sleep(max(0.0, min(0.002, waiting[0].arrival - now)))
            continue
        progressed = False
        for e in engines.values():
            if e.busy is not None:
                segs, ev = e.busy
                if not ev.query():
                    continue
                e.busy = None
                for q in {id(s[0]): s[0] for s in segs}.values():
                    if q.done_cts == q.n_cts:
                        done.append(q)
                        in_use -= q.footprint
                        admitted.remove(q)
                        e.queue.remove(q)
            if e.queue:
                limit = min(round_cts.get(e.log_n, 32) if round_cts else 32, e.ctx.max_batch)
                segs, used = [], 0
                # "srpt": the queries with the fewest ciphertexts left first (ties by arrival),
                # so small queries do not wait behind a large one; "fifo": in admission order
                order = e.queue if policy == "fifo" else sorted(e.queue, key=lambda q: (q.n_cts - q.next_ct, q.arrival))
                for q in order:
                    if used >= limit:
                        break
                    n = min(q.n_cts - q.next_ct, limit - used)
                    if n <= 0:
                        continue
                    segs.append((q, q.next_ct, n))
                    q.next_ct += n
                    used += n
                if segs:
                    e.launch_round(segs)
                    progressed = True
        if not progressed:
            time.sleep(0.0005)
    torch.cuda.synchronize()
    for q in pending:
        q.latency_ms = start_ev.elapsed_time(q.done_event) - q.arrival * 1e3
    lat = np.array([q.latency_ms for q in pending])
    makespan = max(start_ev.elapsed_time(q.done_event) for q in pending) / 1e3
    rows = sum(q.rows for q in pending)
    return {
        "mode": mode,
        "queries": len(pending),
        "rejected": len(rejected),
        "rows": rows,
        "makespan_s": makespan,
        "rows_per_s": rows / makespan,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
    }


def check(queries, engines):
    bad = 0
    for q in queries:
        e = engines[q.log_n]
        got = e.ctx.decrypt(e.s, q.result)[0]
        exp = expected(q)
        bad += int(any(int(v) != exp for v in got))
    return bad


def poisson_arrivals(queries, rate: float, seed: int = 0):
    g = synth.rng(seed, 79, synth.SLOTS, 0)
    t = 0.0
    for q in queries:
        t += g.exponential(1.0 / rate)
        q.arrival = t


def run_mix(n_queries: int = 24, rings=(14, 15, 16), rows_lo: int = 1 << 10, rows_hi: int = 1 << 12,
            load: float = 0.8, round_cts_16: int = 16, seed: int = 0, log=print, policy: str = "srpt") -> dict:
    """A bounded serving run: the mix's columns are encrypted first; the batched capacity is
    measured with every query present at time 0; then arrivals are Poisson at `load` times that
    capacity, served batched and then plain (one at a time).  Every result is checked against
    the plaintext query."""
    rings = list(rings)
    engines = {r: Engine(r, *RING_CHAINS[r], seed=seed) for r in rings}
    qs = make_queries(n_queries, rings, rows_lo, rows_hi, rate=0.0, seed=seed, filter_ring=max(rings))
    prepare(qs, engines, seed=seed)
    log(f"[serve] {len(qs)} queries, {sum(q.rows for q in qs)} rows, encrypted")
    round_cts = {r: round_cts_16 << (16 - r) for r in rings}
    for q in qs:
        q.arrival = 0.0
    cap = serve(qs, engines, mode="batched", round_cts=round_cts, policy=policy)
    rate = load * len(qs) / cap["makespan_s"]
    poisson_arrivals(qs, rate, seed)
    release_cache(engines)
    batched = serve(qs, engines, mode="batched", round_cts=round_cts, policy=policy)
    bad = check(qs, engines)
    log(f"[serve] batched: p50 {batched['p50_ms']:.0f} ms, p99 {batched['p99_ms']:.0f} ms, "
        f"{batched['rows_per_s']:.0f} rows/s")
    release_cache(engines)
    plain = serve(qs, engines, mode="plain")
    bad += check(qs, engines)
    log(f"[serve] plain: p50 {plain['p50_ms']:.0f} ms, p99 {plain['p99_ms']:.0f} ms, {plain['rows_per_s']:.0f} rows/s")
    chains = {str(r): {"L": RING_CHAINS[r][0], "K": RING_CHAINS[r][1], "ntt_split": engines[r].ntt_split,
                       **security_estimate(r, *RING_CHAINS[r])} for r in rings}
    out = {"queries": len(qs), "rows": sum(q.rows for q in qs), "rows_lo": rows_lo, "rows_hi": rows_hi,
           "load_of_batched_capacity": load, "arrival_rate_qps": rate, "batched_capacity_rows_per_s": cap["rows_per_s"],
           "policy": policy, "batched": batched, "plain": plain, "wrong_results": bad, "chains": chains}
    del engines
    release_cache({})
    return out


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="served filter-and-aggregate queries on one GPU")
    ap.add_argument("--rings", default="14,15,16", help="log2 N of the rings in the mix")
    ap.add_argument("--queries", type=int, default=24)
    ap.add_argument("--rows-lo", type=int, default=1 << 10)
    ap.add_argument("--rows-hi", type=int, default=1 << 14)
    ap.add_argument("--load", type=float, default=0.8, help="offered load as a fraction of the batched capacity")
    ap.add_argument("--round-cts", type=int, default=16, help="ciphertexts per round at N = 2^16 (scaled by N)")
    ap.add_argument("--policy", choices=("srpt", "fifo"), default="srpt",
                    help="order in which a round takes the queued queries' ciphertexts")
    args = ap.parse_args(argv)
    rings = [int(x) for x in args.rings.split(",")]
    out = run_mix(args.queries, rings, args.rows_lo, args.rows_hi, args.load, args.round_cts, policy=args.policy)
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
