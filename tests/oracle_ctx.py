"""Small oracle contexts shared by the CPU tests (seeded; no GPU)."""
import functools

from oracle import bgv as B
from oracle.params import Params
from paper_2604_19890_amd import synth

WORKLOAD_TEST = 90


class Ctx:
    def __init__(self, logN, p, r, L, K, steps=(), conj=False, seed=0):
        self.P = Params(logN, p, r, L, K)
        self.seed = seed
        self.s = synth.ternary(self.P.N, seed, WORKLOAD_TEST)
        n_keys = 1 + len(steps) + (1 if conj else 0)
        self.key_rand = [synth.key_randomness(self.P.primes, self.P.N, self.P.dnum, seed, WORKLOAD_TEST, i)
                         for i in range(n_keys)]
        self.keys = B.keygen(self.P, self.s, self.key_rand, steps=steps, with_conj=conj)
        self._n = 0

    def enc(self, slots, idx=None):
        if idx is None:
            self._n += 1
            idx = 1000 + self._n
        c1, e = synth.encryption_randomness(self.P.q, self.P.N, self.seed, WORKLOAD_TEST, idx)
        return B.encrypt(self.P, self.s, slots, c1, e)

    def dec(self, ct):
        vals, nonconst, _ = B.decrypt(self.P, self.s, ct)
        assert not nonconst.any()
        return [int(v) for v in vals]


@functools.lru_cache(maxsize=None)
def tiny5():
    return Ctx(4, 5, 2, 12, 1, steps=(1,), conj=True)


@functools.lru_cache(maxsize=None)
def tiny5_r3():
    """r = 3 (t = 125): Algorithm 3 with G_{5,3} and G_{5,2}; the chain covers less_than's depth."""
    return Ctx(4, 5, 3, 17, 1)


@functools.lru_cache(maxsize=None)
def tiny5_r4():
    """r = 4 (t = 625): G_{5,4}, G_{5,3}, G_{5,2}."""
    return Ctx(4, 5, 4, 26, 1)


@functools.lru_cache(maxsize=None)
def tiny37_r4():
    """p = 37, r = 4 (Table 6's setting, t = 37^4): G_{37,4} of degree 109."""
    return Ctx(4, 37, 4, 40, 1)


@functools.lru_cache(maxsize=None)
def tiny17():
    return Ctx(5, 17, 2, 18, 1, steps=(1, 2), conj=True)


@functools.lru_cache(maxsize=None)
def hybrid17():
    """Digits of two primes (alpha = K = 2) to exercise multi-prime base conversion."""
    return Ctx(5, 17, 2, 7, 2, steps=(1,), conj=True)


@functools.lru_cache(maxsize=None)
def p257():
    """The benchmark's plaintext modulus 257^2 with its chain (30 + 6 primes) on the smallest
    ring that holds all 128 slots (N = 2^8, two coefficients per slot)."""
    return Ctx(8, 257, 2, 30, 6)


@functools.lru_cache(maxsize=None)
def and5():
    """p = 5 with two spare primes for the conjunction of up to four predicates."""
    return Ctx(4, 5, 2, 14, 1)
