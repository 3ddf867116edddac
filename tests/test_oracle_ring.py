"""Pins for the oracle's exact ring kernels (schoolbook product, NTT by definition)."""
import numpy as np
import pytest

from oracle import _ring as R
from oracle.params import find_primes, min_primitive_root_2n


def _rand(N, q, seed):
    g = np.random.default_rng(seed)
    return g.integers(0, q, size=N, dtype=np.uint64)


@pytest.mark.parametrize("N", [8, 64, 256])
def test_schoolbook_is_a_ring_product(N):
    """Evaluation at any root of X^N + 1 is a ring homomorphism; X^N = -1."""
    q = find_primes(N, 25, 1)[0]
    a, b = _rand(N, q, 1), _rand(N, q, 2)
    c = R.negacyclic_dot(a, b, q)
    psi = min_primitive_root_2n(q, N)
    for e in (1, 3, 2 * N - 1):
        w = pow(psi, e, q)
        ev = lambda v: sum(int(x) * pow(w, i, q) for i, x in enumerate(v)) % q
        assert ev(c) == ev(a) * ev(b) % q
    # multiplying by X shifts with a sign wrap
    x = np.zeros(N, dtype=np.uint64)
    x[1] = 1
    sh = R.negacyclic_dot(a, x, q)
    assert int(sh[0]) == (q - int(a[-1])) % q
    assert np.array_equal(sh[1:], a[:-1])


def test_small_and_selected_products_agree_with_the_full_product():
    N = 128
    q = find_primes(N, 289, 1)[0]
    a = _rand(N, q, 3)
    s = np.random.default_rng(4).integers(-1, 2, size=N)
    full = R.negacyclic_dot(a, np.mod(s, q).astype(np.uint64), q)
    assert np.array_equal(R.negacyclic_mul_small(a, s, q), full)
    idx = np.array([0, 5, N - 1])
    assert np.array_equal(R.negacyclic_dot_at(a, np.mod(s, q).astype(np.uint64), q, idx), full[idx])


@pytest.mark.parametrize("N", [8, 32, 256])
def test_ntt_definition_convolution_theorem_and_inverse(N):
    q = find_primes(N, 66049, 2)[1]
    psi = min_primitive_root_2n(q, N)
    a, b = _rand(N, q, 5), _rand(N, q, 6)
    A, Bh = R.ntt_def(a, q, psi), R.ntt_def(b, q, psi)
    C = R.ntt_def(R.negacyclic_dot(a, b, q), q, psi)
    assert np.array_equal(C, R.mulmod_vec(A, Bh, q))  # negacyclic convolution theorem
    assert np.array_equal(R.intt_def(A, q, psi), a)
    # bit-reversed order: slot j is the evaluation at psi^(2 brv(j) + 1)
    logn = N.bit_length() - 1
    j = 1
    brv = int(format(j, f"0{logn}b")[::-1], 2)
    w = pow(psi, 2 * brv + 1, q)
    assert int(A[j]) == sum(int(x) * pow(w, i, q) for i, x in enumerate(a)) % q
