"""Oracle BGV over R_Q = Z_Q[X]/(X^N + 1) in RNS, coefficient form, exact.

Test infrastructure only (see the package docstring).

A ciphertext is (c0, c1) with c0 + c1*s = m + p^r e (mod Q)  (Background, Eq. 1),
stored as uint64 residues c[poly][i][n] in [0, q_i) for the active primes
q_0..q_{level-1}, together with the current plaintext-modulus exponent t_exp
(t = p^t_exp; DivideByP lowers it by one, ChangeModToP sets it to 1, modulus
raising sets it back to r -- Method, reduction and raising subsections).

Readings of what the paper leaves open:
  * encryption is the symmetric Algorithm 1 with c1 uniform per prime and e from
    the seeded clipped Gaussian; every plaintext and constant is lifted to the
    centered range [-(t-1)/2, (t-1)/2] before it is reduced mod q_i;
  * slot values are constants in Z_{p^r} placed as m(X) = M(X^d), where M
    interpolates the slot values at the slot roots;
  * relinearisation and rotation use hybrid key switching with digits of alpha = K
    primes: ksk_j = (b_j, a_j), b_j = -a_j s + t e_j + [prime in digit j] P s';
    ModUp uses the fast base conversion with [x Qhat^-1] in [0, q); ModDown takes
    w = [u_P t^-1] in [0, p_k), converts it to the q-primes by the same formula and
    subtracts t*w before multiplying by P^-1;
  * modulus switching drops the top prime with w = centered([c_top t^-1]_{q_top}),
    c_i <- (c_i - t w) q_top^-1; a multi-level drop is that step repeated (align);
    drop removes top limbs without rescaling (the noise keeps its size);
  * every ciphertext carries the noise estimate of oracle/noise.py (nz), set by
    each operation from its inputs'.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import _ring as R
from . import noise as NZ
from .params import Params


def centered(x: int, m: int) -> int:
    x %= m
    return x - m if x > (m - 1) // 2 else x


@dataclass
class Ct:
    c: np.ndarray  # uint64 [2][level][N]
    level: int
    t_exp: int
    nz: int = 0  # noise estimate, sixteenths of a bit (0: unknown)

    def copy(self):
        return Ct(self.c.copy(), self.level, self.t_exp, self.nz)


@dataclass
class Triple:
    """A tensor product (d0, d1, d2) before relinearisation."""
    d: np.ndarray  # uint64 [3][level][N]
    level: int
    t_exp: int
    nz: int = 0


# ----------------------------------------------------------------------------- encoding

def _root_matrix(P: Params, t_exp: int, count: int) -> np.ndarray:
    """Z[j][a] = zeta_j^a mod t for a < count (int64; t < 2^31)."""
    t = P.t(t_exp)
    roots = P.slot_roots(t_exp)
    Z = np.empty((P.ell, count), dtype=np.int64)
    for j, z in enumerate(roots):
        v = 1
        for a in range(count):
            Z[j, a] = v
            v = v * z % t
    return Z


def encode(P: Params, slots, t_exp: int) -> np.ndarray:
    """Centered integer coefficients (int64, length N) of the plaintext with the given slots.

    M(Y) = sum_k c_k Y^k interpolates the ell slot values at the slot roots; since the
    roots are all primitive 2*ell-th roots of unity, c_k = ell^-1 sum_j v_j zeta_j^-k.
    """
    t = P.t(t_exp)
    v = np.asarray([int(x) % t for x in slots], dtype=object)
    roots = P.slot_roots(t_exp)
    inv_ell = pow(P.ell, -1, t)
    coeffs = []
    for k in range(P.ell):
        acc = 0
        for j, z in enumerate(roots):
            acc += int(v[j]) * pow(z, -k, t)
        coeffs.append(centered(acc * inv_ell, t))
    m = np.zeros(P.N, dtype=np.int64)
    m[:: P.d] = coeffs
    return m


def decode(P: Params, m_mod_t, t_exp: int):
    """Slot values of a plaintext polynomial (coefficients in [0, t)).

    Slot j is m(X) mod (X^d - zeta_j).  Returns (values, nonconstant flags)."""
    t = P.t(t_exp)
    m = np.asarray(m_mod_t, dtype=np.int64).reshape(P.ell, P.d)  # row a holds m_{a d + b}
    Z = _root_matrix(P, t_exp, P.ell)
    res = (Z @ m) % t  # [ell][d]: residue coefficients of X^b
    vals = res[:, 0].astype(np.uint64)
    nonconst = (res[:, 1:] != 0).any(axis=1)
    return vals, nonconst


# ----------------------------------------------------------------------------- helpers

def _qcol(primes):
    return np.asarray(primes, dtype=np.uint64)[:, None]


def reduce_ints(vals, primes) -> np.ndarray:
    """Signed integer vector (int64 or object) -> residues [len(primes)][N]."""
    out = np.empty((len(primes), len(vals)), dtype=np.uint64)
    for i, q in enumerate(primes):
        if isinstance(vals, np.ndarray) and vals.dtype == np.int64:
            out[i] = np.mod(vals, np.int64(q)).astype(np.uint64)
        else:
            out[i] = np.array([int(x) % q for x in vals], dtype=np.uint64)
    return out


def _small_mul(a_limb, s_small, q):
    return R.negacyclic_mul_small(a_limb, s_small, q)


def poly_square_int(s: np.ndarray) -> np.ndarray:
    """s*s in Z[X]/(X^N+1) for a small integer polynomial (exact int64)."""
    N = len(s)
    full = np.convolve(s.astype(np.int64), s.astype(np.int64))
    out = full[:N].copy()
    out[: N - 1] -= full[N:]
    return out


def automorph_int(s: np.ndarray, g: int) -> np.ndarray:
    """s(X^g) for an integer polynomial."""
    N = len(s)
    out = np.zeros(N, dtype=np.int64)
    for i in range(N):
        e = i * g % (2 * N)
        if e < N:
            out[e] += s[i]
        else:
            out[e - N] -= s[i]
    return out


# ----------------------------------------------------------------------------- enc / dec

def encrypt(P: Params, s, slots, c1, e) -> Ct:
    """Algorithm 1 (symmetric BGV encryption) at the top level L with t = p^r."""
    t = P.t_full
    m = encode(P, slots, P.r)
    me = m + t * np.asarray(e, dtype=np.int64)
    s64 = np.asarray(s, dtype=np.int64)
    c1 = np.asarray(c1, dtype=np.uint64)[: P.L]
    c = np.empty((2, P.L, P.N), dtype=np.uint64)
    base = reduce_ints(me, P.q)
    for i, q in enumerate(P.q):
        c1s = _small_mul(c1[i], s64, q)
        c[0, i] = (base[i] + np.uint64(q) - c1s) % np.uint64(q)
        c[1, i] = c1[i]
    return Ct(c, P.L, P.r, NZ.model(P).fresh)


def phase(P: Params, s, ct: Ct) -> list:
    """Centered integers V = [c0 + c1 s]_{Q_level} (Algorithm 2, before the mod t)."""
    s64 = np.asarray(s, dtype=np.int64)
    qs = P.q[: ct.level]
    Q = 1
    for q in qs:
        Q *= q
    V = np.zeros(P.N, dtype=object)
    for i, q in enumerate(qs):
        vi = (ct.c[0, i] + _small_mul(ct.c[1, i], s64, q)) % np.uint64(q)
        Qh = Q // q
        f = Qh * pow(Qh % q, -1, q)
        V = V + vi.astype(object) * f
    half = Q // 2
    return [int(x) % Q - Q if int(x) % Q > half else int(x) % Q for x in V]


def decrypt(P: Params, s, ct: Ct):
    """Algorithm 2: m = (c0 + c1 s mod Q) mod p^t_exp, then slot decoding.

    Returns (slot values, nonconstant-slot flags, noise bits)."""
    V = phase(P, s, ct)
    t = P.t(ct.t_exp)
    m = [v % t for v in V]
    vals, nonconst = decode(P, m, ct.t_exp)
    mx = max(abs(v) for v in V)
    return vals, nonconst, mx.bit_length()


# ----------------------------------------------------------------------------- linear ops

def _check_pair(a: Ct, b: Ct):
    if a.level != b.level:
        raise ValueError("level mismatch")
    if a.t_exp != b.t_exp:
        raise ValueError("plaintext modulus mismatch")


def add(P: Params, a: Ct, b: Ct) -> Ct:
    _check_pair(a, b)
    q = _qcol(P.q[: a.level])
    return Ct((a.c + b.c) % q, a.level, a.t_exp, NZ.add(a.nz, b.nz))


def add_many(P: Params, cts) -> Ct:
    """The sum of ciphertexts of one level and plaintext modulus, as one sum of n terms:
    its estimate bounds n terms by the largest (a + lgc(n)), not by a chain of pairwise
    additions, each of which would add at least a sixteenth of a bit."""
    acc = cts[0]
    for x in cts[1:]:
        _check_pair(acc, x)
    q = _qcol(P.q[: acc.level])
    tot = acc.c
    for x in cts[1:]:
        tot = (tot + x.c) % q
    nz = NZ.sum_of(max(x.nz for x in cts), len(cts)) if all(NZ.known(x.nz) for x in cts) else 0
    return Ct(tot, acc.level, acc.t_exp, nz)


def sub(P: Params, a: Ct, b: Ct) -> Ct:
    _check_pair(a, b)
    q = _qcol(P.q[: a.level])
    return Ct((a.c + (q - b.c)) % q, a.level, a.t_exp, NZ.add(a.nz, b.nz))


def neg(P: Params, a: Ct) -> Ct:
    q = _qcol(P.q[: a.level])
    return Ct((q - a.c) % q, a.level, a.t_exp, a.nz)


def mul_scalar(P: Params, a: Ct, c: int) -> Ct:
    t = P.t(a.t_exp)
    cc = centered(c, t)
    out = np.empty_like(a.c)
    for i, q in enumerate(P.q[: a.level]):
        for k in range(2):
            out[k, i] = R.mulmod_scalar(a.c[k, i], cc % q, q)
    return Ct(out, a.level, a.t_exp, NZ.scalar(a.nz, cc))


def add_const(P: Params, a: Ct, c: int) -> Ct:
    """Add the constant c to every slot: the plaintext of an all-c vector is the constant polynomial c."""
    t = P.t(a.t_exp)
    cc = centered(c, t)
    out = a.c.copy()
    for i, q in enumerate(P.q[: a.level]):
        out[0, i, 0] = (int(out[0, i, 0]) + cc) % q
    return Ct(out, a.level, a.t_exp, NZ.add_const(a.nz, cc))


def divide_by_p(P: Params, a: Ct) -> Ct:
    """DivideByP: multiply by p^-1 mod each q_i and lower t from p^k to p^(k-1)."""
    if a.t_exp < 2:
        raise ValueError("DivideByP needs t = p^k with k >= 2")
    out = np.empty_like(a.c)
    for i, q in enumerate(P.q[: a.level]):
        pinv = pow(P.p, -1, q)
        for k in range(2):
            out[k, i] = R.mulmod_scalar(a.c[k, i], pinv, q)
    return Ct(out, a.level, a.t_exp - 1, NZ.divide_by_p(NZ.model(P), a.nz))


def change_mod_to_p(P: Params, a: Ct) -> Ct:
    """ChangeModToP: only the plaintext modulus tag changes (Lemma 4)."""
    return Ct(a.c.copy(), a.level, 1, a.nz)


def raise_tag(P: Params, a: Ct) -> Ct:
    """First half of modulus raising: the plaintext modulus tag becomes p^r."""
    return Ct(a.c.copy(), a.level, P.r, a.nz)


# ----------------------------------------------------------------------------- modulus switching

def mod_switch(P: Params, a: Ct) -> Ct:
    """Drop the top prime: w = centered([c_top t^-1]_{q_top}); c_i <- (c_i - t w) q_top^-1 mod q_i."""
    lv = a.level
    if lv < 2:
        raise ValueError("cannot drop below one prime")
    qt = P.q[lv - 1]
    t = P.t(a.t_exp)
    tinv = pow(t, -1, qt)
    out = np.empty((2, lv - 1, P.N), dtype=np.uint64)
    for k in range(2):
        wt = R.mulmod_scalar(a.c[k, lv - 1], tinv, qt).astype(np.int64)
        w = np.where(wt > (qt - 1) // 2, wt - np.int64(qt), wt)  # centered
        for i, q in enumerate(P.q[: lv - 1]):
            wi = np.mod(w, np.int64(q)).astype(np.uint64)
            tw = R.mulmod_scalar(wi, t % q, q)
            diff = (a.c[k, i] + np.uint64(q) - tw) % np.uint64(q)
            out[k, i] = R.mulmod_scalar(diff, pow(qt, -1, q), q)
    return Ct(out, lv - 1, a.t_exp, NZ.switch(NZ.model(P), a.nz, a.t_exp))


def drop(P: Params, a: Ct, level: int) -> Ct:
    """The ciphertext modulo its first `level` primes, without rescaling: c0 + c1 s = m + t e
    holds modulo every divisor of the modulus, and the primes are 1 mod t, so the limbs above
    `level` are simply removed (the noise keeps its size)."""
    if level > a.level or level < 1:
        raise ValueError("cannot raise a level")
    return Ct(a.c[:, :level, :].copy(), level, a.t_exp, a.nz)


def align(P: Params, a: Ct, level: int) -> Ct:
    """Sequential single-prime drops down to `level`."""
    if level > a.level:
        raise ValueError("cannot raise a level")
    while a.level > level:
        a = mod_switch(P, a)
    return a


# ----------------------------------------------------------------------------- key switching

@dataclass
class SwitchKey:
    b: np.ndarray  # uint64 [dnum][L+K][N]
    a: np.ndarray  # uint64 [dnum][L+K][N]


def keygen_switch(P: Params, s, s_prime, a_rand, e_rand) -> SwitchKey:
    """b_j = -a_j s + t e_j + [prime in digit j] P s'  over all L+K primes."""
    s64 = np.asarray(s, dtype=np.int64)
    sp = np.asarray(s_prime, dtype=np.int64)
    Pprod = 1
    for pk in P.P:
        Pprod *= pk
    dn = P.dnum
    full_digits = P.digits(P.L)
    b = np.empty((dn, len(P.primes), P.N), dtype=np.uint64)
    a = np.asarray(a_rand, dtype=np.uint64)[:dn].copy()
    for j in range(dn):
        te = P.t_full * np.asarray(e_rand[j], dtype=np.int64)
        for m, q in enumerate(P.primes):
            val = (np.mod(te, np.int64(q)).astype(np.uint64) + np.uint64(q)
                   - _small_mul(a[j, m], s64, q)) % np.uint64(q)
            if m < P.L and m in full_digits[j]:
                ps = R.mulmod_scalar(np.mod(sp, np.int64(q)).astype(np.uint64), Pprod % q, q)
                val = (val + ps) % np.uint64(q)
            b[j, m] = val
    return SwitchKey(b, a)


def mod_up(P: Params, x: np.ndarray, level: int, digit: list) -> np.ndarray:
    """Fast base conversion of one digit to all primes of Q_level and P (coefficient form).

    Returns y [level + K][N]; rows of the digit's own primes are copies of x."""
    targets = list(P.q[:level]) + list(P.P)
    y = np.empty((len(targets), P.N), dtype=np.uint64)
    dq = [P.q[i] for i in digit]
    scaled = []
    for i, qi in zip(digit, dq):
        qh = 1
        for qq in dq:
            if qq != qi:
                qh *= qq
        scaled.append((R.mulmod_scalar(x[i], pow(qh % qi, -1, qi), qi), qh))
    for m, qm in enumerate(targets):
        if m < level and m in digit:
            y[m] = x[m]
            continue
        acc = np.zeros(P.N, dtype=np.uint64)
        for v, qh in scaled:
            acc = (acc + R.mulmod_scalar(v % np.uint64(qm), qh % qm, qm)) % np.uint64(qm)
        y[m] = acc
    return y


def mod_down(P: Params, u: np.ndarray, level: int, t: int) -> np.ndarray:
    """(u - delta) * P^-1 on the q-primes, delta = t * FBC_{P->Q}([u_P t^-1]_P)."""
    K = len(P.P)
    Pprod = 1
    for pk in P.P:
        Pprod *= pk
    scaled = []
    for k, pk in enumerate(P.P):
        w = R.mulmod_scalar(u[level + k], pow(t, -1, pk), pk)
        ph = Pprod // pk
        scaled.append((R.mulmod_scalar(w, pow(ph % pk, -1, pk), pk), ph))
    out = np.empty((level, P.N), dtype=np.uint64)
    for i, qi in enumerate(P.q[:level]):
        acc = np.zeros(P.N, dtype=np.uint64)
        for v, ph in scaled:
            acc = (acc + R.mulmod_scalar(v % np.uint64(qi), ph % qi, qi)) % np.uint64(qi)
        delta = R.mulmod_scalar(acc, t % qi, qi)
        diff = (u[i] + np.uint64(qi) - delta) % np.uint64(qi)
        out[i] = R.mulmod_scalar(diff, pow(Pprod % qi, -1, qi), qi)
    assert K == len(scaled)
    return out


def key_switch(P: Params, x: np.ndarray, key: SwitchKey, level: int, t_exp: int):
    """Hybrid key switching of x [level][N] (coefficient form) -> (u0, u1) [level][N]."""
    digits = P.digits(level)
    ups = [mod_up(P, x, level, dg) for dg in digits]
    key_rows = list(range(level)) + [P.L + k for k in range(len(P.P))]
    u = np.empty((2, level + len(P.P), P.N), dtype=np.uint64)
    for m, row in enumerate(key_rows):
        q = P.primes[row]
        A = np.stack([ups[j][m] for j in range(len(digits))])
        for c, kk in enumerate((key.b, key.a)):
            B = np.stack([kk[j, row] for j in range(len(digits))])
            u[c, m] = R.negacyclic_dot(A, B, q)
    t = P.t(t_exp)
    return mod_down(P, u[0], level, t), mod_down(P, u[1], level, t)


def tensor(P: Params, a: Ct, b: Ct) -> Triple:
    _check_pair(a, b)
    lv = a.level
    d = np.empty((3, lv, P.N), dtype=np.uint64)
    for i, q in enumerate(P.q[:lv]):
        d[0, i] = R.negacyclic_dot(a.c[0, i], b.c[0, i], q)
        d[1, i] = R.negacyclic_dot(np.stack([a.c[0, i], a.c[1, i]]), np.stack([b.c[1, i], b.c[0, i]]), q)
        d[2, i] = R.negacyclic_dot(a.c[1, i], b.c[1, i], q)
    return Triple(d, lv, a.t_exp, NZ.tensor(NZ.model(P), a.nz, b.nz))


def add_tensor(P: Params, d: Triple, e: Triple, level: int) -> Triple:
    """Sum of two tensor-product triples [3][level][N] (component-wise, mod every q_i)."""
    return Triple((d.d + e.d) % _qcol(P.q[:level]), level, d.t_exp, NZ.add(d.nz, e.nz))


def add_to_triple(P: Params, d: Triple, x: Ct) -> Triple:
    """(d0 + c0, d1 + c1, d2): the triple then decrypts to its product plus x's message (both at
    the triple's level and plaintext modulus)."""
    if x.level != d.level or x.t_exp != d.t_exp:
        raise ValueError("level or plaintext modulus mismatch")
    q = _qcol(P.q[: d.level])
    out = d.d.copy()
    out[0] = (out[0] + x.c[0]) % q
    out[1] = (out[1] + x.c[1]) % q
    return Triple(out, d.level, d.t_exp, NZ.add(d.nz, x.nz))


def relin(P: Params, rk: SwitchKey, d: Triple, level: int, t_exp: int) -> Ct:
    """Relinearisation of a triple (d0, d1, d2): (d0 + u0, d1 + u1) with (u0, u1) the key
    switch of d2 (no modulus switch inside)."""
    u0, u1 = key_switch(P, d.d[2], rk, level, t_exp)
    q = _qcol(P.q[:level])
    return Ct(np.stack([(d.d[0] + u0) % q, (d.d[1] + u1) % q]), level, t_exp,
              NZ.key_switch(NZ.model(P), d.nz, t_exp, level))


def mul_relin(P: Params, rk: SwitchKey, a: Ct, b: Ct) -> Ct:
    """Tensor product and relinearisation (no modulus switch inside)."""
    return relin(P, rk, tensor(P, a, b), a.level, a.t_exp)


# ----------------------------------------------------------------------------- automorphisms

def galois_elt(P: Params, step) -> int:
    """X -> X^g: g = 5^step mod 2N for a row rotation, 2N-1 for the row swap ('conj')."""
    if step == "conj":
        return 2 * P.N - 1
    return pow(5, int(step), 2 * P.N)


def automorph_limbs(P: Params, x: np.ndarray, g: int, primes) -> np.ndarray:
    N = P.N
    idx = (np.arange(N, dtype=np.int64) * g) % (2 * N)
    out = np.empty_like(x)
    for i, q in enumerate(primes):
        v = x[i]
        negv = (np.uint64(q) - v) % np.uint64(q)
        lo = idx < N
        out[i, idx[lo]] = v[lo]
        out[i, idx[~lo] - N] = negv[~lo]
    return out


def rotate(P: Params, gk: dict, a: Ct, step) -> Ct:
    g = galois_elt(P, step)
    primes = P.q[: a.level]
    c0 = automorph_limbs(P, a.c[0], g, primes)
    c1 = automorph_limbs(P, a.c[1], g, primes)
    u0, u1 = key_switch(P, c1, gk[g], a.level, a.t_exp)
    q = _qcol(primes)
    return Ct(np.stack([(c0 + u0) % q, u1]), a.level, a.t_exp, NZ.key_switch(NZ.model(P), a.nz, a.t_exp, a.level))


# ----------------------------------------------------------------------------- keys

@dataclass
class Keys:
    relin: SwitchKey
    galois: dict  # g -> SwitchKey


def keygen(P: Params, s, key_rand, steps=(), with_conj=False) -> Keys:
    """key_rand[i] = (a, e) for key i: 0 = relinearisation, then each step, then the row swap."""
    s64 = np.asarray(s, dtype=np.int64)
    a, e = key_rand[0]
    relin = keygen_switch(P, s64, poly_square_int(s64), a, e)
    gal = {}
    order = list(steps) + (["conj"] if with_conj else [])
    for i, st in enumerate(order):
        g = galois_elt(P, st)
        a, e = key_rand[1 + i]
        gal[g] = keygen_switch(P, s64, automorph_int(s64, g), a, e)
    return Keys(relin, gal)


# ----------------------------------------------------------------------------- sampled outputs
# The same computations restricted to a set of output coefficient indices, for
# checks at ring sizes where the full schoolbook products take too long.  Every
# step is coefficient-wise except the ring products, which are evaluated only at
# the requested indices; inputs that feed a product are still used in full.

def mod_down_cols(P: Params, u: np.ndarray, level: int, t: int) -> np.ndarray:
    """mod_down applied to selected columns: u [level+K][S] -> [level][S] (columns are independent)."""
    return mod_down(_SubP(P, u.shape[1]), u, level, t)


class _SubP:
    """View of Params with N replaced by a column count (coefficient-wise steps only)."""

    def __init__(self, P, ncols):
        self._P = P
        self.N = ncols

    def __getattr__(self, k):
        return getattr(self._P, k)


def key_switch_at(P: Params, x: np.ndarray, key: SwitchKey, level: int, t_exp: int, idx) -> tuple:
    """key_switch(x) evaluated only at coefficient indices idx (x is the full [level][N] input)."""
    digits = P.digits(level)
    ups = [mod_up(P, x, level, dg) for dg in digits]
    key_rows = list(range(level)) + [P.L + k for k in range(len(P.P))]
    idx = np.asarray(idx, dtype=np.int64)
    u = np.empty((2, level + len(P.P), len(idx)), dtype=np.uint64)
    for m, row in enumerate(key_rows):
        q = P.primes[row]
        A = np.stack([ups[j][m] for j in range(len(digits))])
        for c, kk in enumerate((key.b, key.a)):
            B = np.stack([kk[j, row] for j in range(len(digits))])
            u[c, m] = R.negacyclic_dot_at(A, B, q, idx)
    t = P.t(t_exp)
    return mod_down_cols(P, u[0], level, t), mod_down_cols(P, u[1], level, t)


def mul_relin_at(P: Params, rk: SwitchKey, a: Ct, b: Ct, idx) -> np.ndarray:
    """mul_relin(a, b) at coefficient indices idx: array [2][level][len(idx)]."""
    _check_pair(a, b)
    lv = a.level
    idx = np.asarray(idx, dtype=np.int64)
    d2 = np.empty((lv, P.N), dtype=np.uint64)
    d01 = np.empty((2, lv, len(idx)), dtype=np.uint64)
    for i, q in enumerate(P.q[:lv]):
        d2[i] = R.negacyclic_dot(a.c[1, i], b.c[1, i], q)
        d01[0, i] = R.negacyclic_dot_at(a.c[0, i], b.c[0, i], q, idx)
        d01[1, i] = R.negacyclic_dot_at(np.stack([a.c[0, i], a.c[1, i]]), np.stack([b.c[1, i], b.c[0, i]]), q, idx)
    u0, u1 = key_switch_at(P, d2, rk, lv, a.t_exp, idx)
    q = _qcol(P.q[:lv])
    return np.stack([(d01[0] + u0) % q, (d01[1] + u1) % q])


def rotate_at(P: Params, gk: dict, a: Ct, step, idx) -> np.ndarray:
    g = galois_elt(P, step)
    primes = P.q[: a.level]
    c0 = automorph_limbs(P, a.c[0], g, primes)
    c1 = automorph_limbs(P, a.c[1], g, primes)
    idx = np.asarray(idx, dtype=np.int64)
    u0, u1 = key_switch_at(P, c1, gk[g], a.level, a.t_exp, idx)
    q = _qcol(primes)
    return np.stack([(c0[:, idx] + u0) % q, u1])


def encrypt_at(P: Params, s, slots, c1, e, idx) -> np.ndarray:
    """c0 of Algorithm 1 at coefficient indices idx: [L][len(idx)] (c1 is the input itself)."""
    t = P.t_full
    m = encode(P, slots, P.r)
    me = m + t * np.asarray(e, dtype=np.int64)
    sm = np.asarray(s, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty((P.L, len(idx)), dtype=np.uint64)
    for i, q in enumerate(P.q):
        s_res = np.mod(sm, np.int64(q)).astype(np.uint64)
        c1s = R.negacyclic_dot_at(np.asarray(c1[i], dtype=np.uint64), s_res, q, idx)
        out[i] = (np.mod(me[idx], np.int64(q)).astype(np.uint64) + np.uint64(q) - c1s) % np.uint64(q)
    return out


def sampled(P: Params, ct: Ct, idx) -> Ct:
    """The columns idx of a ciphertext, as a ciphertext over a ring of len(idx) coefficients
    (valid input for the coefficient-wise steps: add, mod_switch, mul_scalar)."""
    return Ct(np.ascontiguousarray(ct.c[:, :, idx]), ct.level, ct.t_exp)


def mod_switch_cols(P: Params, ct: Ct) -> Ct:
    """mod_switch on a column-sampled ciphertext (coefficient-wise)."""
    return mod_switch(_SubP(P, ct.c.shape[2]), ct)
