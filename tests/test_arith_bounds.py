"""Exactness of the library's binary64 modular arithmetic at the extremes (CPU).

The kernels carry residues below 2^50 as doubles and reduce lazily; their correctness
rests on stated bounds (a Barrett product within (3m/8 + 1/2) q for a multiplicand of
magnitude m q, Cooley-Tukey register steps below 7.1 q, Gentleman-Sande steps below 4 q with
multiplicands below 8 q, exact split sums of small-coefficient combinations).  This test
compiles the library's own arithmetic headers (modarith.hpp, ntt_stages.hpp) for the host
with g++ and checks those statements against exact 128-bit integer arithmetic on extremal
operands (+-q, q - 1, (q - 1)/2, the largest and smallest moduli) and random ones, for every
prime of the benchmark's chain and the moduli at both ends of [2^49, 2^50)."""
import json
import os
import subprocess

import pytest

from oracle.params import Params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "arith_bounds.cpp")
INC = os.path.join(ROOT, "paper_2604_19890_amd", "csrc")


def _largest_prime_below(n):
    def is_prime(m):
        if m % 2 == 0:
            return False
        d, s = m - 1, 0
        while d % 2 == 0:
            d //= 2
            s += 1
        for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
            x = pow(a, d, m)
            if x in (1, m - 1):
                continue
            for _ in range(s - 1):
                x = x * x % m
                if x == m - 1:
                    break
            else:
                return False
        return True
    m = n - 1
    while not is_prime(m):
        m -= 1
    return m


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("arith") / "arith_bounds")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", INC, "-o", exe, SRC])
    return exe


def test_modular_arithmetic_bounds_hold_at_the_extremes(checker):
    moduli = set(Params(16, 257, 2, 30, 6).primes) | set(Params(12, 17, 2, 18, 1).primes)
    moduli |= {_largest_prime_below(1 << 50), (1 << 50) - 1, (1 << 49) + 1}
    r = subprocess.run([checker, *map(str, sorted(moduli))], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    rows = [json.loads(line) for line in r.stdout.splitlines()]
    assert len(rows) == len(moduli)
    for row in rows:
        assert row["failures"] == 0
        # the stated bounds (the checker fails on any violation; these are the headroom figures)
        assert all(m <= 3 * f / 8 + 0.5 for m, f in zip(row["mul_max"], (1.0, 1.9, 3.1, 4.8, 8.0)))
        assert row["ct_max"][3] < 7.1 and max(row["gs_max"]) < 4.0 and row["gs_mult_max"] < 8.0
        assert row["red_max_over_q"] <= 0.5 + 2.0 / row["q"]
