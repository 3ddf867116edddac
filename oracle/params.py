"""Oracle parameters: RNS primes, NTT roots and the slot structure of X^N + 1 mod p^r.

Test infrastructure only (see the package docstring).

Ring: the scheme's R_Q = Z_Q[X]/Phi_m(X) (Background, BGV subsection) taken with
m = 2N a power of two, so Phi_m = X^N + 1.  Plaintexts live in R_{p^r}; the slot
decomposition Phi_m = prod F_i mod p^r with ell = phi(m)/d factors of degree
d = Ord(m, p) is the one the paper describes for packing.  For p = 1 mod 4 the
factors are X^d - zeta_j with zeta_j running over the primitive 2*ell-th roots of
unity of Z_{p^r}, ell = 2^(v2(p-1)-1), d = N/ell.

Readings fixed here (where the paper is silent):
  * ciphertext primes are 50-bit primes q = 1 mod lcm(2N, p^r), listed in
    descending order from 2^50; the first L are q_0..q_{L-1}, the next K are the
    special primes of hybrid key switching;
  * the NTT root of a prime q is the smallest primitive 2N-th root of unity mod q;
  * slot roots: zeta is the Teichmuller lift to Z_{p^r} of the smallest integer in
    [2, p) of multiplicative order 2*ell mod p; slot index rho*ell/2 + c holds the
    root zeta^{(-1)^rho * 5^c mod 2 ell}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (the twelve prime bases)."""
    if n < 2:
        return False
    for b in _MR_BASES:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def find_primes(N: int, t: int, count: int, bits: int = 50) -> list[int]:
    """The first `count` primes below 2^bits (descending) that are 1 mod lcm(2N, t)."""
    M = math.lcm(2 * N, t)
    x = ((2 ** bits - 2) // M) * M + 1
    out = []
    while len(out) < count:
        if x < 2 ** (bits - 1):
            raise ValueError("not enough primes of the requested size")
        if is_prime(x):
            out.append(x)
        x -= M
    return out


def min_primitive_root_2n(q: int, N: int) -> int:
    """Smallest primitive 2N-th root of unity mod q (q = 1 mod 2N)."""
    e = (q - 1) // (2 * N)
    x = 2
    while True:
        c = pow(x, e, q)
        if pow(c, N, q) == q - 1:
            break
        x += 1
    best = c
    c2 = c * c % q
    w = c
    for _ in range(N - 1):
        w = w * c2 % q
        if w < best:
            best = w
    return best


def v2(n: int) -> int:
    k = 0
    while n % 2 == 0:
        n //= 2
        k += 1
    return k


@dataclass
class Params:
    logN: int
    p: int
    r: int
    L: int
    K: int
    # polynomial evaluation schedule ("fast" or "basic"; see space.eval_poly)
    schedule: str = "fast"
    N: int = field(init=False)
    t_full: int = field(init=False)
    alpha: int = field(init=False)
    q: list = field(init=False)
    P: list = field(init=False)
    primes: list = field(init=False)
    ell: int = field(init=False)
    d: int = field(init=False)
    zeta: int = field(init=False)
    slot_exps: list = field(init=False)

    def __post_init__(self):
        self.N = 1 << self.logN
        self.t_full = self.p ** self.r
        self.alpha = self.K
        if self.p % 4 != 1:
            raise ValueError("only p = 1 mod 4 is supported by the power-of-two ring")
        allp = find_primes(self.N, self.t_full, self.L + self.K)
        self.q = allp[: self.L]
        self.P = allp[self.L:]
        self.primes = allp
        v = v2(self.p - 1)
        self.ell = 1 << (v - 1)
        if 2 * self.N < (1 << v):
            raise ValueError("ring too small for this p")
        self.d = self.N // self.ell
        zb = next(z for z in range(2, self.p)
                  if pow(z, self.ell, self.p) == self.p - 1)
        self.zeta = pow(zb, self.p ** (self.r - 1), self.t_full)
        two_l = 2 * self.ell
        half = self.ell // 2
        exps = []
        for rho in range(2):
            for c in range(half):
                e = pow(5, c, two_l)
                exps.append(e if rho == 0 else (two_l - e) % two_l)
        self.slot_exps = exps
        self._psi = {}

    def t(self, t_exp: int) -> int:
        return self.p ** t_exp

    def psi(self, prime: int) -> int:
        if prime not in self._psi:
            self._psi[prime] = min_primitive_root_2n(prime, self.N)
        return self._psi[prime]

    def digits(self, level: int) -> list:
        """Digit index sets of hybrid key switching at a level (alpha primes each)."""
        a = self.alpha
        return [list(range(j * a, min((j + 1) * a, level))) for j in range((level + a - 1) // a)]

    @property
    def dnum(self) -> int:
        return (self.L + self.alpha - 1) // self.alpha

    def slot_roots(self, t_exp: int) -> list:
        t = self.t(t_exp)
        z = self.zeta % t
        return [pow(z, e, t) for e in self.slot_exps]
