"""Oracle polynomial evaluation and the space-switching composites.

Test infrastructure only (see the package docstring).

Polynomial evaluation follows the baby-step/giant-step form of Paterson-Stockmeyer
(Theorem 2).  The paper does not spell out the schedule; the reading fixed here,
which decides every ciphertext bit, is:

  degree D, k = smallest power of two with 2 k^2 >= D + 1, g = ceil((D+1)/k);
  baby powers x^i (2 <= i <= k) and giant powers y^j (y = x^k, 2 <= j <= g-1) by the
  power rule: h = 2^floor(log2 i); x^i = x^(i/2) x^(i/2) if i = h, else x^h x^(i-h)
  (in the fast schedule the powers of two and the giants first, then the other baby
  powers the inner sums need, each at the level its consumers need: _late_babies);
  every product is: bring both operands to the lower level (below), relinearised
  product, one modulus switch;
  inner sums I_j = sum_{i=1}^{k-1} c_{jk+i} x^i over nonzero coefficients only,
  each power first brought to the lowest level among the powers used, scalar
  products accumulated in increasing i, then the constant c_{jk} added;
  an inner sum with no power term contributes c_{jk} y^j as a scalar product;
  outer sum over j = 1..g-1 in increasing j (each term I_j * y^j a product as
  above), operands brought to the lower level before each addition, I_0 added last
  (in the fast schedule the constant inner sums' terms c_jk y^j and I_0 join the summed outer
  products before their one switch).

Bringing an operand to a lower level: in the basic schedule by single-prime modulus
switches; in the fast schedule by its noise estimate (oracle/noise.py): while the
estimate is more than SLACK above the floor a switch leaves, one switch of the top
prime, then the remaining limbs are dropped without rescaling.  Dropping leaves the
noise as it is, which is then at most SLACK above what switches would leave.

Composites (Method section, any r):
  space_reduce = Algorithm 3: balanced base-p digits by recursion (the lift polynomial
                 G_{p,e} gives the lowest digit, DivideByP of the rest recurses), each
                 digit finally read modulo p;
  compare      = Algorithm 4: a fold over the digits from the most significant down,
                 state (lt, eq) absorbing each digit's (LT_i, EQ_i), EQ_i = 1 - x_i^(p-1)
                 with the power from the power rule;
  space_raise  = RaiseModToP2R: plaintext modulus back to p^r, then G_{p,r}.
"""
from __future__ import annotations

from . import bgv as B
from . import noise as NZ
from . import polys


class Counter:
    def __init__(self):
        self.mul = 0
        self.max_depth = 0


def _lower(P, x, level):
    """x brought to `level` (see the module docstring)."""
    if x.level == level:
        return x
    if P.schedule == "basic" or not NZ.known(x.nz):
        return B.align(P, x, level)
    floor = NZ.model(P).floor[x.t_exp]
    while x.level > level and x.nz > floor + NZ.SLACK:
        x = B.mod_switch(P, x)
    return B.drop(P, x, level) if x.level > level else x


def _mul(P, keys, a, b, cnt=None):
    """a b relinearised and switched down one prime, each operand first brought to the lower
    level."""
    lv = min(a.level, b.level)
    a = _lower(P, a, lv)
    b = _lower(P, b, lv)
    r = B.mul_relin(P, keys.relin, a, b)
    if cnt is not None:
        cnt.mul += 1
    return B.mod_switch(P, r)


def _lazy_level(pairs):
    return min(min(a.level, b.level) for a, b in pairs)


def _lazy_products(P, keys, pairs, cnt=None, addends=()):
    """sum_j a_j b_j relinearised once: every operand brought to the lowest level among the
    pairs, the tensor products summed, one key switch of the summed d2, one modulus switch.
    Addends (k, x): k x for each, in their order, x at that level or above and brought down by
    dropping limbs, join (d0, d1) before the key switch, so the one modulus switch also divides
    their noise."""
    lv = _lazy_level(pairs)
    acc = None
    for a, b in pairs:
        d = B.tensor(P, _lower(P, a, lv), _lower(P, b, lv))
        acc = d if acc is None else B.add_tensor(P, acc, d, lv)
        if cnt is not None:
            cnt.mul += 1
    for k, x in addends:
        xd = B.drop(P, x, lv)
        acc = B.add_to_triple(P, acc, xd if k == 1 else B.mul_scalar(P, xd, k))
    return B.mod_switch(P, B.relin(P, keys.relin, acc, lv, pairs[0][0].t_exp))


def _add(P, a, b):
    lv = min(a.level, b.level)
    return B.add(P, _lower(P, a, lv), _lower(P, b, lv))


def odd_structured(c, D: int) -> bool:
    """True when D >= 3 and every coefficient at an even index 2 <= i < D is zero: the
    polynomial is odd apart from its constant and leading terms (G_{p,e} for odd p is odd,
    Section IV's parity property; F_LT has odd terms and x^(p-1))."""
    return D >= 3 and all(c[i] == 0 for i in range(2, D, 2))


def bsgs_shape(D: int, odd: bool = False):
    """Paterson-Stockmeyer split (Theorem 2): k baby powers, g giant steps in y = x^k.

    Dense polynomials: k = smallest power of two with 2k^2 >= D+1.  Odd-structured ones
    need only the odd baby powers, which halves the baby steps; the balance point moves to
    k = smallest power of two with k^2 >= D+1 (a constant or a leading term at a multiple
    of k lands in an inner sum as a constant)."""
    k = 1
    if odd:
        while k * k < D + 1:
            k *= 2
    else:
        while 2 * k * k < D + 1:
            k *= 2
    g = -(-(D + 1) // k)
    return k, g


def _power_rule(table, i, P, keys, cnt):
    """x^i = x^(i/2) x^(i/2) for i a power of two, else x^h x^(i-h) (h the largest power of two
    below i)."""
    if i in table:
        return table[i]
    h = 1 << (i.bit_length() - 1)
    if i == h:
        half = _power_rule(table, i // 2, P, keys, cnt)
        table[i] = _mul(P, keys, half, half, cnt)
    else:
        table[i] = _mul(P, keys, _power_rule(table, h, P, keys, cnt),
                        _power_rule(table, i - h, P, keys, cnt), cnt)
    return table[i]


def _late_babies(P, keys, baby, giant, k, g, coef, cnt):
    """Fast schedule: the baby powers other than the powers of two, each formed at the level
    its consumers need rather than as high as its operands allow.

    The needed powers are the exponents the inner sums use, closed under the power rule's
    operands.  The outer products meet at F, the lowest level among the giant powers of the
    non-constant inner sums; a power x^i = x^h x^(i-h) (h the largest power of two below i)
    is wanted at level F for the inner sums, and at one level above each power it is the
    second operand of.  It is formed by a product at one level above that (or lower, if an
    operand is lower), its operands brought down first."""
    used = {i for j in range(g) for i in range(1, k) if coef(j * k + i) != 0}
    need = set()

    def close(i):
        if i <= 1 or i in need:
            return
        need.add(i)
        h = 1 << (i.bit_length() - 1)
        if i == h:
            close(i // 2)
        else:
            close(h)
            close(i - h)

    for i in used | {k}:
        close(i)
    late = sorted(i for i in need if i & (i - 1))
    prods = [j for j in range(1, g) if any(coef(j * k + i) != 0 for i in range(1, k))]
    if not prods:
        for i in late:
            _power_rule(baby, i, P, keys, cnt)
        return
    F = min(giant[j].level for j in prods)
    want = {i: F for i in late}
    for i in reversed(late):
        second = i - (1 << (i.bit_length() - 1))
        if second in want:
            want[second] = max(want[second], want[i] + 1)
    for i in late:
        h = 1 << (i.bit_length() - 1)
        a, b = baby[h], baby[i - h]
        lv = min(want[i] + 1, a.level, b.level)
        baby[i] = _mul(P, keys, _lower(P, a, lv), _lower(P, b, lv), cnt)


def power(P, keys, x, e, cnt=None):
    """x^e by the power rule (e >= 1)."""
    table = {1: x}
    return _power_rule(table, e, P, keys, cnt)


def eval_poly(P, keys, x, coeffs, cnt=None, parity=True):
    """Evaluate sum_i coeffs[i] x^i (coefficients mod t = p^t_exp of x) by Paterson-Stockmeyer
    (Theorem 2) in the schedule P.schedule.

    "fast": with parity (the default) an odd-structured polynomial takes the odd split of
    bsgs_shape; the outer products I_j y^j are relinearised once, after their tensor products
    are summed; the inner sums are formed at the level where those products meet; operands are
    lowered by their noise estimates.
    "basic": the dense split for every polynomial; each inner sum at the lowest level among
    its powers; in increasing j, I_j y^j as one product (_mul) or c_jk y^j, added to the
    running sum at the lower level; then I_0."""
    basic = P.schedule == "basic"
    t = P.t(x.t_exp)
    c = [int(v) % t for v in coeffs]
    D = len(c) - 1
    while D > 0 and c[D] == 0:
        D -= 1
    k, g = bsgs_shape(D, (not basic) and parity and odd_structured(c, D))

    def coef(n):
        return c[n] if n <= D else 0

    baby = {1: x}
    if basic:
        for i in range(2, k + 1):
            _power_rule(baby, i, P, keys, cnt)
    else:
        # the powers of two up to x^k (y) by squaring, then the giant powers
        i = 2
        while i <= k:
            _power_rule(baby, i, P, keys, cnt)
            i *= 2
    giant = {1: baby[k]}
    for j in range(2, g):
        _power_rule(giant, j, P, keys, cnt)
    if not basic:
        _late_babies(P, keys, baby, giant, k, g, coef, cnt)

    # every inner sum is formed at the level where the outer products meet (the lowest
    # level among the non-constant I_j and their y^j), or at its own lowest level if lower
    used_all = [[i for i in range(1, k) if coef(j * k + i) != 0] for j in range(g)]
    own = [min(baby[i].level for i in u) if u else None for u in used_all]
    prods = [j for j in range(1, g) if used_all[j]]
    meet = min(min(own[j], giant[j].level) for j in prods) if prods and not basic else None
    inner = []
    for j in range(g):
        used = used_all[j]
        const = coef(j * k)
        if not used:
            inner.append(("const", const))
            continue
        lv = own[j] if meet is None else min(own[j], meet)
        acc = None
        for i in used:
            xi = _lower(P, baby[i], lv)
            term = B.mul_scalar(P, xi, coef(j * k + i))
            acc = term if acc is None else B.add(P, acc, term)
        if const != 0:
            acc = B.add_const(P, acc, const)
        inner.append(("ct", acc))

    result = None
    if basic:
        # in increasing j: I_j y^j as one product, or c_jk y^j, added at the lower level
        for j in range(1, g):
            kind, v = inner[j]
            if kind == "ct":
                term = _mul(P, keys, v, giant[j], cnt)
            elif v != 0:
                term = B.mul_scalar(P, giant[j], v)
            else:
                continue
            result = term if result is None else _add(P, result, term)
    else:
        # the products I_j y^j, relinearised once together; the scalar multiples c_jk y^j of
        # constant inner sums (increasing j), then I_0, join them before the switch when they
        # are at that level or above, otherwise they are added after it
        pairs = [(v, giant[j]) for j, (kind, v) in enumerate(inner) if j >= 1 and kind == "ct"]
        scalars = [(v, giant[j]) for j, (kind, v) in enumerate(inner) if j >= 1 and kind == "const" and v != 0]
        if pairs:
            lv = _lazy_level(pairs)
            add = [(k, y) for k, y in scalars if y.level >= lv]
            scalars = [(k, y) for k, y in scalars if y.level < lv]
            kind0, v0 = inner[0]
            if kind0 == "ct" and v0.level >= lv:
                add.append((1, v0))
                inner[0] = ("folded", None)
            result = _lazy_products(P, keys, pairs, cnt, addends=add)
        else:
            result = None
        for k, y in scalars:
            term = B.mul_scalar(P, y, k)
            result = term if result is None else _add(P, result, term)
    kind, v = inner[0]
    if kind == "const":
        if result is None:
            raise ValueError("constant polynomial: nothing to evaluate")
        if v != 0:
            result = B.add_const(P, result, v)
    elif kind == "ct":
        result = v if result is None else _add(P, result, v)
    return result


def space_reduce(P, keys, a, cnt=None):
    """Algorithm 3: the balanced base-p digits of a value tagged t = p^e, least significant
    first, each tagged t = p.

    The lowest digit is G_{p,e} of the value (Lemma 3: the polynomial keeps the residue mod p
    and lands on its balanced representative mod p^e).  Subtracting it leaves a multiple of p;
    dividing by p leaves the value of the remaining digits, tagged p^(e-1), whose digits follow
    the same way, down to a value tagged p, which is the top digit itself.  Each digit is
    finally read modulo p alone."""
    def digits(b):
        e = b.t_exp
        if e == 1:
            return [b]
        low = eval_poly(P, keys, b, polys.g_poly(P.p, e), cnt)
        rest = B.divide_by_p(P, B.sub(P, _lower(P, b, low.level), low))
        return [low] + digits(rest)

    return [B.change_mod_to_p(P, d) for d in digits(a)]


def _eq_digit(P, keys, x, cnt):
    y = power(P, keys, x, P.p - 1, cnt)
    return B.add_const(P, B.neg(P, y), 1)


def _one_minus(P, ct):
    return B.add_const(P, B.neg(P, ct), 1)


def compare(P, keys, digits, op="lt", cnt=None):
    """Algorithm 4 over the digits (given least significant first).

    A value is below zero exactly when its most significant nonzero balanced digit is.  Reading
    the digits from the top down, the state (lt, eq) says whether the digits read so far are
    below zero, and whether they are all zero; the next digit with indicators (LT_i, EQ_i)
    moves it to (lt + eq LT_i, eq EQ_i), and the top digit's indicators start it.  LT_i is the
    digit polynomial F_LT (F_GT for 'gt') at the digit, EQ_i = 1 - x_i^(p-1) (Fermat).  The
    last digit's eq is never formed.

    op: 'lt', 'gt', 'eq' (the fold's eq alone), and the complements of the comparison
    subsection: 'ge' = 1 - LT, 'le' = 1 - GT, 'neq' = 1 - EQ."""
    if op in ("ge", "le", "neq"):
        base = {"ge": "lt", "le": "gt", "neq": "eq"}[op]
        return _one_minus(P, compare(P, keys, digits, base, cnt))
    top = len(digits) - 1
    if op == "eq":
        eq = _eq_digit(P, keys, digits[top], cnt)
        for x in reversed(digits[:top]):
            eq = _mul(P, keys, eq, _eq_digit(P, keys, x, cnt), cnt)
        return eq
    f = polys.f_lt(P.p) if op == "lt" else polys.f_gt(P.p)
    lt = eval_poly(P, keys, digits[top], f, cnt)
    eq = _eq_digit(P, keys, digits[top], cnt) if top > 0 else None
    for i in range(top - 1, -1, -1):
        lt = _add(P, lt, _mul(P, keys, eq, eval_poly(P, keys, digits[i], f, cnt), cnt))
        if i > 0:
            eq = _mul(P, keys, eq, _eq_digit(P, keys, digits[i], cnt), cnt)
    return lt


def space_raise(P, keys, a, cnt=None):
    """RaiseModToP2R: tag t = p^r, then G_{p,r} clears the higher digits."""
    x = B.raise_tag(P, a)
    return eval_poly(P, keys, x, polys.g_poly(P.p, P.r), cnt)


def less_than(P, keys, x, y, cnt=None):
    """[x < y] in the number space (t = p^r), through reduce -> compare -> raise."""
    d = B.sub(P, x, y) if y is not None else x
    return space_raise(P, keys, compare(P, keys, space_reduce(P, keys, d, cnt), "lt", cnt), cnt)


def masked_product(P, keys, x, y, v, cnt=None):
    """v * [x < y]  (the tiny primitive pipeline)."""
    return _mul(P, keys, less_than(P, keys, x, y, cnt), v, cnt)


def relu(P, keys, x, cnt=None):
    """x * (1 - [x < 0])."""
    lt = less_than(P, keys, x, None, cnt)
    return _mul(P, keys, x, B.add_const(P, B.neg(P, lt), 1), cnt)


def _product_at(P, keys, b, c, level, cnt=None):
    """b c formed where it is consumed: by a product one level above `level` (the level of
    the factor it meets; lower if an operand is lower), its operands brought down first.  In
    the basic schedule, at the operands' own level."""
    if P.schedule == "basic":
        return _mul(P, keys, b, c, cnt)
    lv = min(level + 1, b.level, c.level)
    return _mul(P, keys, _lower(P, b, lv), _lower(P, c, lv), cnt)


def filter_product(P, keys, a, tq, b, c, cnt=None):
    """[a < tq] * (b * c) for one ciphertext of rows; b * c is formed at the predicate's level."""
    m = less_than(P, keys, a, tq, cnt)
    return _mul(P, keys, m, _product_at(P, keys, b, c, m.level, cnt), cnt)


def filter_and_product(P, keys, preds, b, c, cnt=None):
    """[every predicate holds] * (b * c) for one ciphertext of rows: a conjunction of the
    comparison subsection's predicates, as range filters need (lo <= a AND a < hi).

    preds: (column, threshold, op) triples; predicate i is op applied to the digits of
    column - threshold ('lt' is [column < threshold], 'ge' is [column >= threshold], ...).  Each
    0/1 result stays in the digit space (t = p); the conjunction is their product there, taken
    as a balanced tree over the predicates in their order (pairs (0, 1), (2, 3), .., then pairs of
    those); it is raised once to t = p^r and multiplied by b * c, formed at that level."""
    bits = [compare(P, keys, space_reduce(P, keys, B.sub(P, col, thr), cnt), op, cnt) for col, thr, op in preds]
    while len(bits) > 1:
        paired = [_mul(P, keys, bits[i], bits[i + 1], cnt) for i in range(0, len(bits) - 1, 2)]
        if len(bits) % 2:
            paired.append(bits[-1])
        bits = paired
    m = space_raise(P, keys, bits[0], cnt)
    return _mul(P, keys, m, _product_at(P, keys, b, c, m.level, cnt), cnt)


def rotate_and_sum(P, keys, ct):
    """Every slot ends up holding the sum of all slots: row rotations by 2^i, then the row swap."""
    i = 1
    while i < P.ell // 2:
        ct = B.add(P, ct, B.rotate(P, keys.galois, ct, i))
        i *= 2
    return B.add(P, ct, B.rotate(P, keys.galois, ct, "conj"))
