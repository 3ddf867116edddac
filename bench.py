"""Benchmark: encrypted filter + SUM rows/s on one MI355X.

Workload: SUM(b * c WHERE a < t) over rows packed 128 per ciphertext in the ring
N = 2^16 with plaintext modulus 257^2 (columns a, b, c uniform 16-bit values,
threshold t uniform in [0, 2^16) as one encrypted broadcast ciphertext), 30 ciphertext
primes + 6 special primes.  A step runs the whole query on one batch of
`--cts` ciphertexts per column: a - t, space_reduce, compare, space_raise, the
b*c product, the masked product, the batch sum and rotate-and-sum, with every
input already resident in HBM.  value = rows per second of the batched form.

Also reported on the same line:
  plain      -- the same query with one ciphertext per call (every launch covers one ciphertext)
  ntt        -- forward NTT GB/s on the query's ciphertext shape (16 N bytes per limb)
  roofline   -- the NTT passes (the most frequent kernels) against the 8 TB/s HBM peak
  cpu_baseline -- the CPU oracle on a bounded sample (one product at N = 2^16), scaled
                  to rows/s by the query's count of schoolbook limb products.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LOG_N, P_, R_, L_, K_ = 16, 257, 2, 30, 6
HBM_PEAK_GBS = 8000.0

# HBM traffic of the forward NTT (both passes) on 960 limbs of N = 2^16, per pass, from
# `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` runs of `bench.py --ntt-only --cts 16
# --steps 3` (profiles/ntt_n65536_960limbs.md).  In the same runs a 480 MiB device
# copy reads FETCH_SIZE = 245782 KiB and WRITE_SIZE = 491520 KiB, so FETCH_SIZE counts half
# the bytes moved (scale 2.0) and WRITE_SIZE all of them (1.0).  The figures belong to the
# NTT sources they were taken on (hash below) and are reported only while those are unchanged.
NTT_COUNTERS = {
    "sources_sha256": "49663687e55e64cff561abe8304328f19f325ee18438e09bfb8417e8aa6b8316",
    "limbs": 960,
    "fetch_kib": [246089, 253498],
    "write_kib": [491520, 491520],
    "fetch_scale": 2.0,
    "write_scale": 1.0,
}


def ntt_sources_sha256():
    h = hashlib.sha256()
    for name in ("ntt.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2604_19890_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def ntt_traffic_bytes(limbs):
    """Counter-measured HBM bytes of one forward NTT over `limbs` limbs, or None when the NTT
    sources differ from the ones the counters were read on."""
    c = NTT_COUNTERS
    if ntt_sources_sha256() != c["sources_sha256"]:
        return None
    per_transform = 1024 * (sum(c["fetch_kib"]) * c["fetch_scale"] + sum(c["write_kib"]) * c["write_scale"])
    return per_transform * limbs / c["limbs"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(args):
    import torch
    from paper_2604_19890_amd import bgv as G
    from paper_2604_19890_amd import synth

    ctx = G.Context(LOG_N, P_, R_, L_, K_)
    N, ell = ctx.N, ctx.slots
    wl = 2
    s = synth.ternary(N, args.seed, wl)
    steps = [1 << i for i in range(6)]  # 1..32: rotate-and-sum over a row of 64 slots
    n_keys = 1 + len(steps) + 1
    t0 = time.time()
    ka = np.empty((n_keys, ctx.dnum, ctx.L + ctx.K, N), dtype=np.uint64)
    ke = np.empty((n_keys, ctx.dnum, N), dtype=np.int32)
    for i in range(n_keys):
        ka[i], ke[i] = synth.key_randomness(ctx.primes, N, ctx.dnum, args.seed, wl, i)
    keys = ctx.keygen(s, ka, ke, steps=steps, with_conj=True)
    del ka, ke
    log(f"[bench] keys {keys.bytes / 2**20:.0f} MiB in {time.time() - t0:.1f}s")

    B = args.cts
    g = synth.rng(args.seed, wl, synth.SLOTS, 0)
    cols = {k: g.integers(0, 1 << 16, size=(B, ell), dtype=np.uint64) for k in "abc"}
    thr = int(g.integers(0, 1 << 16))
    if args.bits < 16:  # the filter column and threshold on a narrower range
        cols["a"] >>= np.uint64(16 - args.bits)
        thr >>= 16 - args.bits

    def enc(rows, base):
        c1 = np.empty((len(rows), ctx.L, N), dtype=np.uint64)
        e = np.empty((len(rows), N), dtype=np.int32)
        for i in range(len(rows)):
            c1[i], e[i] = synth.encryption_randomness(ctx.primes[:ctx.L], N, args.seed, wl, base + i)
        return ctx.encrypt(s, rows, c1, e)

    t0 = time.time()
    cts = {k: enc(cols[k], 100000 * (j + 1)) for j, k in enumerate("abc")}
    cts["t"] = enc(np.full((1, ell), thr, dtype=np.uint64), 900000)
    torch.cuda.synchronize()
    log(f"[bench] encrypted 3 x {B} + 1 ciphertexts in {time.time() - t0:.1f}s")
    return ctx, keys, s, cols, thr, cts


def expected_sum(cols, thr, t=P_ ** R_):
    a, b, c = (cols[k].astype(np.int64) for k in "abc")
    d = (a - thr) % t
    lt = d > (t - 1) // 2  # centered(a - thr) < 0
    return int((b * c * lt).sum() % t)


def sql_agreement(cols, thr, t=P_ ** R_):
    """How the circuit's predicate (centered a - thr < 0 in Z_t) compares with the integer
    predicate a < thr: the fraction of rows where they agree (all rows when |a - thr| <=
    (t - 1) / 2, e.g. 15-bit values), and whether the SUM equals the integer query's."""
    a, b, c = (cols[k].astype(np.int64) for k in "abc")
    circ = ((a - thr) % t) > (t - 1) // 2
    sql = a < thr
    return {"rows_agree": float((circ == sql).mean()),
            "sum_equals_sql": int((b * c * sql).sum() % t) == expected_sum(cols, thr, t)}


def time_batched(ctx, keys, cts, steps, warmup):
    import torch
    for _ in range(warmup):
        ctx.filter_sum(keys, cts["a"], cts["t"], cts["b"], cts["c"])
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    out = None
    for i in range(steps):
        out = ctx.filter_sum(keys, cts["a"], cts["t"], cts["b"], cts["c"])
        log(f"[bench] step {i + 1}/{steps} enqueued")
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3, out


def time_plain(ctx, keys, cts, n_plain):
    """One ciphertext per call: the same query, looping over the first n_plain rows-ciphertexts."""
    import torch
    from paper_2604_19890_amd.bgv import Ct

    N = ctx.N

    def one(name, i):
        x = cts[name]
        w = x.tensor.numel() // x.n
        return Ct(x.tensor[i * w:(i + 1) * w], 1, x.level, x.t_exp)

    def run():
        acc = None
        for i in range(n_plain):
            bc = ctx.mul(keys, one("b", i), one("c", i))
            lt = ctx.less_than(keys, one("a", i), cts["t"])
            prod = ctx.mul(keys, lt, bc)
            acc = prod if acc is None else ctx.add(acc, prod)
        return ctx.rotate_sum(keys, acc)

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def time_graph(ctx, keys, cts, steps):
    """The batched step captured once as a hipGraph and replayed."""
    import torch
    out = ctx.empty(1, 1)
    ctx.filter_sum(keys, cts["a"], cts["t"], cts["b"], cts["c"], out=out)  # eager run: tables, scratch
    torch.cuda.synchronize()
    ctx.capture_begin()
    ctx.filter_sum(keys, cts["a"], cts["t"], cts["b"], cts["c"], out=out)
    graph = ctx.capture_end()
    graph.launch()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        graph.launch()
    stop.record()
    torch.cuda.synchronize()
    del graph
    return start.elapsed_time(stop) / 1e3 / steps


def time_ntt(ctx, n_cts, reps=20, warm_s=1.0):
    """Forward NTT over n_cts ciphertexts at the top level: per-NTT time with HIP events on the
    context's stream, after `warm_s` seconds of untimed transforms, which bring the clocks to their
    sustained level (ten warm-up transforms leave the time 5-10% above it)."""
    import torch
    limbs = n_cts * 2 * ctx.L
    x = torch.randint(0, 1 << 49, (limbs * ctx.N,), dtype=torch.int64, device="cuda")
    t0 = time.perf_counter()
    while True:
        for _ in range(10):
            ctx.ntt(x, n_cts * 2, ctx.L)
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= warm_s:
            break
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        ctx.ntt(x, n_cts * 2, ctx.L)
    stop.record()
    torch.cuda.synchronize()
    per = start.elapsed_time(stop) / 1e3 / reps
    algo_bytes = 16.0 * ctx.N * limbs
    return per, algo_bytes, limbs


def ntt_only(args):
    """Forward NTT over --cts ciphertexts (2 x 30 limbs each) and a device copy of the same
    number of bytes, reps times each: the run the hardware counters are read on."""
    import torch
    from paper_2604_19890_amd import bgv as G
    ctx = G.Context(LOG_N, P_, R_, L_, K_)
    limbs = args.cts * 2 * ctx.L
    x = torch.randint(0, 1 << 49, (limbs * ctx.N,), dtype=torch.int64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.steps):
        ctx.ntt(x, args.cts * 2, ctx.L)
        y.copy_(x)
    torch.cuda.synchronize()
    per, algo_bytes, limbs = time_ntt(ctx, args.cts, reps=args.steps, warm_s=0.0)
    log(f"[bench] ntt-only: {limbs} limbs, {algo_bytes / 2**30:.3f} GiB algorithmic per transform, "
        f"copy of {x.numel() * 8 / 2**30:.3f} GiB; {per * 1e6:.1f} us per transform")


# ----------------------------------------------------------------------------- CPU oracle baseline

def limb_products_per_query_ct():
    """Schoolbook limb products the oracle performs per ciphertext of the query, by replaying the
    oracle's own schedule on level-only stand-ins (a cost model; no arithmetic)."""
    import oracle.bgv as OB
    import oracle.space as OS
    from oracle.params import Params

    P = Params(LOG_N, P_, R_, L_, K_)
    count = {"prod": 0}

    class Fake:
        def __init__(self, level, t_exp):
            self.level, self.t_exp = level, t_exp

    def mul_relin(P_, rk, a, b):
        lv = a.level
        dn = len(P.digits(lv))
        count["prod"] += 4 * lv + 2 * dn * (lv + K_)
        return Fake(lv, a.t_exp)

    def tensor(P_, a, b):
        count["prod"] += 4 * a.level
        return Fake(a.level, a.t_exp)

    def relin(P_, rk, d, level, t_exp):
        count["prod"] += 2 * len(P.digits(level)) * (level + K_)
        return Fake(level, t_exp)

    def rotate(P_, gk, a, step):
        lv = a.level
        count["prod"] += 2 * len(P.digits(lv)) * (lv + K_)
        return Fake(lv, a.t_exp)

    saved = {k: getattr(OB, k) for k in ("mul_relin", "mod_switch", "add", "sub", "neg", "mul_scalar",
                                        "add_const", "divide_by_p", "change_mod_to_p", "raise_tag", "rotate",
                                        "tensor", "relin", "add_tensor", "drop")}
    try:
        OB.mul_relin = mul_relin
        OB.tensor = tensor
        OB.relin = relin
        OB.add_tensor = lambda P_, d, e, level: d
        OB.rotate = rotate
        OB.mod_switch = lambda P_, a: Fake(a.level - 1, a.t_exp)
        OB.drop = lambda P_, a, level: Fake(level, a.t_exp)
        OB.add = lambda P_, a, b: Fake(a.level, a.t_exp)
        OB.sub = lambda P_, a, b: Fake(a.level, a.t_exp)
        OB.neg = lambda P_, a: Fake(a.level, a.t_exp)
        OB.mul_scalar = lambda P_, a, c: Fake(a.level, a.t_exp)
        OB.add_const = lambda P_, a, c: Fake(a.level, a.t_exp)
        OB.divide_by_p = lambda P_, a: Fake(a.level, a.t_exp - 1)
        OB.change_mod_to_p = lambda P_, a: Fake(a.level, 1)
        OB.raise_tag = lambda P_, a: Fake(a.level, P.r)
        x = lambda: Fake(L_, R_)
        Kfake = type("K", (), {"relin": None, "galois": None})()
        OS.filter_product(P, Kfake, x(), x(), x(), x())
        per_ct = count["prod"]
        count["prod"] = 0
        OS.rotate_and_sum(P, Kfake, Fake(1, R_))
        tail = count["prod"]
    finally:
        for k, v in saved.items():
            setattr(OB, k, v)
    return per_ct, tail


def cpu_baseline(n_cts):
    from oracle import bgv as OB
    from oracle.params import Params
    from paper_2604_19890_amd import synth

    lv = 2
    P = Params(LOG_N, P_, R_, lv, K_)
    s = synth.ternary_hw(P.N, 120, 0, 3)
    kr = [synth.key_randomness(P.primes, P.N, P.dnum, 0, 3, 0)]
    keys = OB.keygen(P, s, kr)

    def enc(i):
        c1, e = synth.encryption_randomness(P.q, P.N, 0, 3, i)
        return OB.encrypt(P, s, list(range(P.ell)), c1, e)

    a, b = enc(1), enc(2)
    t0 = time.perf_counter()
    OB.mul_relin(P, keys.relin, a, b)
    dt = time.perf_counter() - t0
    sample_prods = 4 * lv + 2 * len(P.digits(lv)) * (lv + K_)
    per_prod = dt / sample_prods
    per_ct, tail = limb_products_per_query_ct()
    t_query = per_prod * (per_ct * n_cts + tail)
    rows = n_cts * P.ell
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": rows / t_query,
        "unit": "rows/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"one oracle mul_relin at N=2^16, level {lv}, K={K_} ({sample_prods} schoolbook limb products, "
                   f"{dt:.1f}s); scaled by the oracle schedule's {per_ct} limb products per 128-row ciphertext "
                   f"(+{tail} for the final rotate-and-sum) over {n_cts} ciphertexts"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cts", type=int, default=32, help="ciphertexts per column per step (128 rows each)")
    ap.add_argument("--plain", type=int, default=2, help="ciphertexts timed in the plain form")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true", help="also time the step replayed from a hipGraph")
    ap.add_argument("--ntt-only", action="store_true",
                    help="only the forward NTT at the query shape and a copy of the same bytes (for counters)")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-basic-schedule", action="store_true",
                    help="skip timing the query in the basic evaluation schedule")
    ap.add_argument("--no-ntt", action="store_true",
                    help="skip the standalone NTT timing (roofline null), e.g. to profile the query alone")
    ap.add_argument("--bits", type=int, default=16, choices=range(1, 17), metavar="1..16",
                    help="range of the filter column and threshold (16: the workload; 15: the circuit's "
                         "comparison equals the integer one on every row)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; sharding over several GPUs is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if args.ntt_only:
        ntt_only(args)
        return
    ctx, keys, s, cols, thr, cts = setup(args)
    rows = args.cts * ctx.slots

    # the dominant kernel, the forward NTT at the query's ciphertext shape (16 ciphertexts),
    # timed before the query after its own warm-up
    ntt_gbs, ntt_limbs = None, min(args.cts, 16) * 2 * ctx.L
    if not args.no_ntt:
        ntt_s, ntt_bytes, ntt_limbs = time_ntt(ctx, min(args.cts, 16))
        ntt_gbs = ntt_bytes / ntt_s / 1e9
        log(f"[bench] NTT: {ntt_limbs} limbs in {ntt_s * 1e3:.3f} ms = {ntt_gbs:.0f} GB/s")

    elapsed, out = time_batched(ctx, keys, cts, args.steps, args.warmup)
    per_step = elapsed / args.steps
    value = rows / per_step
    log(f"[bench] batched: {per_step * 1e3:.1f} ms/step, {value:.1f} rows/s")
    if not args.no_check:
        got = ctx.decrypt(s, out)[0]
        exp = expected_sum(cols, thr)
        assert all(int(v) == exp for v in got), (got[:4], exp)
        log(f"[bench] decrypted SUM = {exp} in every slot (matches the plaintext query)")

    # the same query in the basic evaluation schedule (one product per outer Paterson-Stockmeyer
    # term, dense split), for comparison with the default schedule timed above
    basic_sched = None
    if not args.no_basic_schedule:
        ctx.set_schedule("basic")
        el, out_p = time_batched(ctx, keys, cts, args.steps, 1)
        ctx.set_schedule("fast")
        if not args.no_check:
            assert all(int(v) == expected_sum(cols, thr) for v in ctx.decrypt(s, out_p)[0])
        basic_sched = {"ms_per_step": el / args.steps * 1e3, "rows_per_s": rows * args.steps / el}
        log(f"[bench] basic schedule: {el / args.steps * 1e3:.1f} ms/step, {rows * args.steps / el:.1f} rows/s")

    t_graph = time_graph(ctx, keys, cts, args.steps) if args.graph else None
    if t_graph:
        log(f"[bench] graph replay: {t_graph * 1e3:.1f} ms/step, {rows / t_graph:.1f} rows/s")
    t_plain = time_plain(ctx, keys, cts, args.plain) if args.plain > 0 else None
    plain_rows = (args.plain * ctx.slots / t_plain) if t_plain else None
    if t_plain:
        log(f"[bench] plain: {t_plain * 1e3:.1f} ms for {args.plain} ciphertexts, {plain_rows:.1f} rows/s")

    traffic = ntt_traffic_bytes(ntt_limbs)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cts)
    line = {
        "metric": "encrypted filter+SUM rows/s @N=2^16 (batched)",
        "value": value,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"filter_sum N=2^16 p=257 r=2 L=30 K=6, {args.cts} ciphertexts x 128 rows per column"
                               + (f", {args.bits}-bit filter column" if args.bits < 16 else ""),
                   "rows_per_step": rows, "parallelism": "batch"},
        "plain_rows_per_s": plain_rows,
        "graph_rows_per_s": (rows / t_graph) if t_graph else None,
        "batched_over_plain": (value / plain_rows) if plain_rows else None,
        "basic_schedule": basic_sched,
        "ntt_gb_per_s": ntt_gbs,
        "roofline": None if ntt_gbs is None else {
                     "bound": "hbm", "achieved": ntt_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ntt_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"k_ntt_pass, forward NTT (two passes) over {ntt_limbs} limbs of N=2^16; "
                               f"achieved = 16 N bytes per limb / transform time; traffic = counter bytes "
                               f"per transform"},
        "cpu_baseline": cpu,
        "sql_agreement": sql_agreement(cols, thr),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
