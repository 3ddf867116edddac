"""Oracle coefficient tables of the digit-space and lifting polynomials.

Test infrastructure only (see the package docstring).

* F_EQ(x, 0) = 1 - x^(p-1) over Z_p (Fermat's little theorem, Theorem 1 and Eq. 2;
  restated for comparison with zero in the Method's comparison subsection).
* F_LT(x, 0) = (p+1)/2 x^(p-1) + sum_{i odd, 1 <= i <= p-2} c_i x^i with
  c_i = sum_{j=1}^{(p-1)/2} j^(p-1-i)  (Method, comparison subsection).
* F_GT(x, 0) = F_LT(-x, 0): GT is obtained the same way as LT.
* G_{p,2}: a polynomial with G(z0 + p z1) = z0 mod p^2 for balanced z0 (Lemma 3).
  The paper defers the construction; the reading used here is the monic form
  G(x) = x^p + p H(x) mod p^2, where H in F_p[x] (degree <= p-1) interpolates
  (z - z^p)/p mod p at every balanced z.  Then G(z) = z mod p^2 on balanced z and
  G'(z) = 0 mod p, which gives Lemma 3's property by Taylor expansion; its degree
  p meets Lemma 3's bound (e-1)(p-1)+1 for e = 2.
* G_{p,e}, e >= 3: lifted from G_{p,e-1} one digit at a time (the reading used here;
  the paper defers to Chen-Han).  With Q(x) = x^p - x, Q(z0 + p y)/p = c(z0) - y (mod p)
  where c(z0) = (z0^p - z0)/p, so Q exposes the high digit y.  If G_k(z0 + p y) =
  z0 + p^k E(z0, y) (mod p^(k+1)), E has degree <= k in y; writing -E(z0, c - u) =
  sum_m e_m(z0) u^m and M_m for the interpolant (degree <= p-1, mod p) of e_m over the
  balanced z0, G_{k+1} = G_k + sum_m p^(k-m) Q^m M_m  (mod p^(k+1)) satisfies Lemma 3's
  property mod p^(k+1) (E is sampled at y = 0..k, so e <= p).  For e = 3 only m <= 1 occurs
  and the degree is 2p - 1, Lemma 3's bound; the construction keeps G odd.
All coefficient lists are ascending (index i is the coefficient of x^i), values in [0, modulus).
"""
from __future__ import annotations

import functools


@functools.lru_cache(maxsize=None)
def _f_eq(p: int) -> tuple:
    c = [0] * p
    c[0] = 1
    c[p - 1] = p - 1
    return tuple(c)


def f_eq(p: int) -> list:
    return list(_f_eq(p))


@functools.lru_cache(maxsize=None)
def _f_lt(p: int) -> tuple:
    c = [0] * p
    c[p - 1] = (p + 1) // 2 % p
    for i in range(1, p - 1, 2):
        c[i] = sum(pow(j, p - 1 - i, p) for j in range(1, (p - 1) // 2 + 1)) % p
    return tuple(c)


def f_lt(p: int) -> list:
    return list(_f_lt(p))


def _poly_mul(a, b, m):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                out[i + j] = (out[i + j] + x * y) % m
    return out


def lagrange(points, values, m):
    """Coefficients of the unique polynomial of degree < len(points) through the points, mod prime m."""
    n = len(points)
    result = [0] * n
    for i, (xi, yi) in enumerate(zip(points, values)):
        if yi % m == 0:
            continue
        num = [1]
        den = 1
        for j, xj in enumerate(points):
            if j != i:
                num = _poly_mul(num, [(-xj) % m, 1], m)
                den = den * (xi - xj) % m
        scale = yi * pow(den, -1, m) % m
        for k in range(n):
            result[k] = (result[k] + scale * num[k]) % m
    return result


@functools.lru_cache(maxsize=None)
def _g_p2(p: int) -> tuple:
    zs = list(range(-(p - 1) // 2, (p - 1) // 2 + 1))
    phi = [((z - z ** p) // p) % p for z in zs]
    H = lagrange([z % p for z in zs], phi, p)
    t = p * p
    G = [(p * h) % t for h in H] + [0]
    G[p] = (G[p] + 1) % t
    return tuple(G)


def f_gt(p: int) -> list:
    """F_GT(x, 0) = [x > 0] on the balanced representatives: F_LT(-x) (the comparison
    subsection derives GT the same way as LT)."""
    return [(c if i % 2 == 0 else -c) % p for i, c in enumerate(f_lt(p))]


def g_p2(p: int) -> list:
    """Coefficients of G_{p,2} mod p^2 (length p + 1)."""
    return list(_g_p2(p))


def _poly_add(a, b, m):
    out = [0] * max(len(a), len(b))
    for i, x in enumerate(a):
        out[i] = x
    for i, x in enumerate(b):
        out[i] = (out[i] + x) % m
    return [v % m for v in out]


def _eval_int(coeffs, x):
    acc = 0
    for c in reversed(coeffs):
        acc = acc * x + c
    return acc


@functools.lru_cache(maxsize=None)
def _g_poly(p: int, e: int) -> tuple:
    if e == 1:
        return (0, 1)  # the identity: digit extraction mod p is the value itself
    if e == 2:
        return _g_p2(p)
    k = e - 1
    if k + 1 > p:
        raise ValueError("the lift samples E(z0, y) at k + 1 distinct y mod p: needs e <= p")
    G = list(_g_poly(p, k))  # Lemma 3's property mod p^k
    mod = p ** e
    h = (p - 1) // 2
    zs = list(range(-h, h + 1))
    Q = [0] * (p + 1)
    Q[1], Q[p] = -1, 1
    # e_m(z0) for every balanced z0: E(z0, y) = (G(z0 + p y) - z0) / p^k mod p sampled at
    # y = 0..k and interpolated (degree <= k), then rewritten in u = c(z0) - y
    em = [[0] * p for _ in range(k + 1)]
    for zi, z in enumerate(zs):
        E = lagrange(list(range(k + 1)),
                     [((_eval_int(G, z + p * y) - z) // p ** k) % p for y in range(k + 1)], p)
        c = ((z ** p - z) // p) % p
        # E(c - u) = sum_j E_j (c - u)^j: expand by the binomial theorem
        for j, Ej in enumerate(E):
            for m in range(j + 1):
                term = Ej * _binom(j, m) * pow(c, j - m, p) * (-1) ** m
                em[m][zi] = (em[m][zi] - term) % p
    out = [v % mod for v in G]
    Qm = [1]  # Q^m
    for m in range(k + 1):
        if any(em[m]):
            M = lagrange([z % p for z in zs], em[m], p)
            term = [(p ** (k - m)) * v for v in _poly_mul_int(Qm, M)]
            out = _poly_add(out, term, mod)
        Qm = _poly_mul_int(Qm, Q)
    while len(out) > 1 and out[-1] == 0:
        out.pop()
    return tuple(out)


def _binom(n, k):
    r = 1
    for i in range(k):
        r = r * (n - i) // (i + 1)
    return r


def _poly_mul_int(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                out[i + j] += x * y
    return out


def g_poly(p: int, e: int) -> list:
    """Coefficients of G_{p,e} mod p^e (Lemma 3): G(z0 + p z1) = z0 mod p^e for balanced z0."""
    return list(_g_poly(p, e))


def eval_mod(coeffs, x: int, m: int) -> int:
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * x + c) % m
    return acc
