"""Pins for the oracle's parameters: primes, NTT roots and the slot structure."""
import math

import numpy as np
import pytest

from oracle.params import Params, find_primes, min_primitive_root_2n


def _sieve(limit):
    s = np.ones(limit + 1, dtype=bool)
    s[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if s[i]:
            s[i * i:: i] = False
    return np.nonzero(s)[0].astype(np.uint64)


SMALL = _sieve(1 << 25)  # every prime below 2^25 > sqrt(2^50)


def _trial_division_prime(n):
    return not np.any(np.uint64(n) % SMALL[SMALL < np.uint64(n)] == 0)


@pytest.mark.parametrize("logN,t,count", [(12, 289, 20), (15, 66049, 20), (16, 66049, 36)])
def test_primes_are_the_descending_ntt_friendly_50bit_primes(logN, t, count):
    N = 1 << logN
    ps = find_primes(N, t, count)
    M = math.lcm(2 * N, t)
    assert ps == sorted(ps, reverse=True)
    for q in ps:
        assert 2 ** 49 <= q < 2 ** 50
        assert q % M == 1
        assert _trial_division_prime(q)
    # nothing skipped: every candidate between consecutive primes (and above the first) is composite
    cand = list(range(ps[0] + M, 2 ** 50, M)) + [x for a, b in zip(ps, ps[1:]) for x in range(b + M, a, M)]
    for x in cand[:400]:
        assert not _trial_division_prime(x)


@pytest.mark.parametrize("N", [16, 64, 1024])
def test_psi_is_the_smallest_primitive_2n_root(N):
    q = find_primes(N, 25, 1)[0]
    psi = min_primitive_root_2n(q, N)
    assert pow(psi, N, q) == q - 1
    # brute force over all primitive 2N-th roots: psi0^(odd) for any primitive root psi0
    g = next(x for x in range(2, 1000) if pow(pow(x, (q - 1) // (2 * N), q), N, q) == q - 1)
    psi0 = pow(g, (q - 1) // (2 * N), q)
    roots = {pow(psi0, e, q) for e in range(1, 2 * N, 2)}
    assert len(roots) == N and psi == min(roots)


def _polymul_mod(a, b, m):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] = (out[i + j] + x * y) % m
    return out


@pytest.mark.parametrize("logN,p,r", [(4, 5, 2), (5, 17, 2), (4, 17, 2), (8, 257, 2), (5, 13, 2)])
def test_slot_factorisation_of_x_n_plus_1(logN, p, r):
    """X^N + 1 = prod_j (X^d - zeta_j) mod p^r with ell = N/d distinct slot roots."""
    P = Params(logN, p, r, 2, 1)
    t = P.t_full
    roots = P.slot_roots(r)
    assert len(set(roots)) == P.ell
    prod = [1]
    for z in roots:
        f = [(-z) % t] + [0] * (P.d - 1) + [1]
        prod = _polymul_mod(prod, f, t)
    expect = [1] + [0] * (P.N - 1) + [1]
    assert prod == expect
    # slot roots are primitive 2*ell-th roots; zeta is a Teichmuller lift (zeta^(p-1) = 1)
    for z in roots:
        assert pow(z, P.ell, t) == t - 1
    assert pow(P.zeta, p - 1, t) == 1
    # d is the multiplicative order of p modulo 2N (the paper's d = Ord(m, p))
    assert min(k for k in range(1, 2 * P.N) if pow(p, k, 2 * P.N) == 1) == P.d
