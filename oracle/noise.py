"""Oracle noise estimate: a bound on the noise of every ciphertext, carried with it.

Test infrastructure only (see the package docstring).

The paper sizes the ciphertext modulus to the depth of the circuit (its parameter
section) and leaves noise management to the library; it gives no noise model.  The
model here is a reading of the standard BGV analysis, stated so that the evaluator
can decide, per operand, whether bringing it to a lower level needs rescaling
switches or only dropping limbs.

Quantity.  For a ciphertext with c0 + c1 s = m + t e (mod Q), the noise is
nu = [c0 + c1 s]_Q (centered, the plaintext included), and the estimate nz is a
bound on log2 of its largest coefficient, in sixteenths of a bit (an integer).  0
means "unknown" (a batch that did not come from this model); an unknown input makes
the result unknown, and an unknown operand is always rescaled.

Bounds (t = p^e of the ciphertext, n = log2 N, alpha = K, Q16 = floor(16 log2) of
the smallest ciphertext prime; "6 sigma" is a high-probability bound on a
coefficient that is a sum of many independent terms):
  fresh encryption    |m| <= t/2 and |t e| <= 19 t  ->  lgc(20 t)
  a + b, a - b        bound of 2^a + 2^b (lsum below)
  k * a (centered k)  a + lgc(|k|)
  a + const k         lsum(a, lgc(|k|))
  DivideByP           a - lgf(p): the noise polynomial itself is divided by p
  ChangeModToP, tag   unchanged (the same polynomial)
  drop limbs          unchanged
  switch floor R(e)   t (tau0 + tau1 s), tau uniform in [-1/2, 1/2], s ternary:
                      6 sigma <= 1.5 t sqrt(N)  ->  lgc(3 t) - 16 + 8 n
  modulus switch      lsum(a - Q16, R(e))
  tensor product      6 sigma of a sum of N products: 2 sqrt(N) 2^a 2^b -> a + b + 8 n + 16
  key switching adds  K(e, l) = lsum(lgc(23 alpha t) + ceil(lgc(dnum_l) / 2) + 8 n,
                                     lgc(3 alpha t) + 8 n)
                      (digits x~_j < alpha Q_j times t e_j over P, 6 sigma with
                      sigma_e = 3.2 and Q_j / P < 2; plus the ModDown rounding
                      t (w0 + w1 s) / P with w < alpha P), dnum_l = ceil(l / alpha)
  relinearise         lsum(tensor, K(e, l));  rotation: lsum(a, K(e, l))
lsum(a, b) = max(a, b) + d(|a - b|) with d a step function above
16 log2(1 + 2^(-|a-b|/16)), so it bounds the sum of the two bounds.

Every result is clamped to at least 1 (a known bound stays known).  The test suite
checks that the estimate bounds the measured noise of the oracle's ciphertexts
through the whole pipeline."""
from __future__ import annotations

import functools

U = 16  # units per bit
SLACK = 4 * U  # an operand within 4 bits of the switch floor is lowered by dropping limbs


def lgc(x: int) -> int:
    """ceil(16 log2 x) for an integer x >= 1, exactly (bit length of x^16 - 1)."""
    return (x ** 16 - 1).bit_length()


def lgf(x: int) -> int:
    """floor(16 log2 x) for an integer x >= 1, exactly."""
    return (x ** 16).bit_length() - 1


def lsum(a: int, b: int) -> int:
    """A bound (sixteenths of a bit) on log2(2^(a/16) + 2^(b/16))."""
    d = abs(a - b)
    if d < 16:
        add = 16  # log2(1 + 2^-x) <= 1 for x >= 0
    elif d < 32:
        add = 10  # <= log2(1.5) = 0.585
    elif d < 48:
        add = 6  # <= log2(1.25) = 0.322
    elif d < 64:
        add = 3  # <= log2(1.125) = 0.170
    elif d < 96:
        add = 2  # <= log2(1.0625) = 0.0875
    else:
        add = 1  # <= log2(1 + 1/64) = 0.0224
    return max(a, b) + add


class Model:
    def __init__(self, logN: int, p: int, r: int, L: int, K: int, q: tuple):
        self.n = logN
        self.p, self.r, self.L, self.alpha = p, r, L, K
        self.fresh = lgc(20 * p ** r)
        self.q16 = lgf(min(q))
        self.lgp = lgf(p)
        self.floor = {e: lgc(3 * p ** e) - U + 8 * logN for e in range(1, r + 1)}
        self.ks = {}
        for e in range(1, r + 1):
            t = p ** e
            for lv in range(1, L + 1):
                dn = -(-lv // K)
                self.ks[e, lv] = lsum(lgc(23 * K * t) + (lgc(dn) + 1) // 2 + 8 * logN, lgc(3 * K * t) + 8 * logN)


@functools.lru_cache(maxsize=None)
def _model(logN, p, r, L, K, q):
    return Model(logN, p, r, L, K, q)


def model(P) -> Model:
    return _model(P.logN, P.p, P.r, P.L, P.K, tuple(P.q))


def known(*xs) -> bool:
    return all(x > 0 for x in xs)


def sum_of(a: int, n: int) -> int:
    """A bound on a sum of n terms, each bounded by 2^(a/16): n 2^(a/16), i.e. a + lgc(n)."""
    return max(1, a + lgc(n)) if known(a) else 0


def add(a: int, b: int) -> int:
    return max(1, lsum(a, b)) if known(a, b) else 0


def scalar(a: int, k: int) -> int:
    """k centered."""
    return max(1, a + (lgc(abs(k)) if k else 0)) if known(a) else 0


def add_const(a: int, k: int) -> int:
    """k centered."""
    return max(1, lsum(a, lgc(abs(k))) if k else a) if known(a) else 0


def divide_by_p(M: Model, a: int) -> int:
    return max(1, a - M.lgp) if known(a) else 0


def switch(M: Model, a: int, t_exp: int) -> int:
    return max(1, lsum(a - M.q16, M.floor[t_exp])) if known(a) else 0


def tensor(M: Model, a: int, b: int) -> int:
    return a + b + 8 * M.n + U if known(a, b) else 0


def key_switch(M: Model, a: int, t_exp: int, level: int) -> int:
    """a plus the noise one key switch at `level` adds (relinearisation, rotation)."""
    return max(1, lsum(a, M.ks[t_exp, level])) if known(a) else 0
