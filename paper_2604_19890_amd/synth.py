"""Seeded synthetic inputs shared by the GPU path, the oracle tests and the benchmark.

This module only draws random numbers; it holds none of the scheme's arithmetic.
Every stream is keyed by ``(seed, workload, purpose, index)`` through NumPy's
``SeedSequence`` so that any consumer can regenerate exactly the same arrays.

Distributions (the reading of the paper's parameter section and of the
workload definitions):

* secret key: uniform ternary coefficients in {-1, 0, 1}
* error: discrete Gaussian, sigma = 3.2, sampled as round-half-even of a normal
  deviate and clipped to [-19, 19]
* uniform ring elements: independent uniform residues in [0, q) for each modulus
  q the caller passes in (the generator never derives moduli itself)
* slot data: uniform integers in a caller-given range, or clipped normals for the
  ReLU workload
"""
from __future__ import annotations

import numpy as np

# purpose tags for stream splitting
SECRET = 1
ERROR = 2
UNIFORM = 3
SLOTS = 4
KEY_A = 5
KEY_E = 6
ENC_C1 = 7
ENC_E = 8
PERM = 9

SIGMA = 3.2
ERROR_CLIP = 19


def rng(seed: int, workload: int, purpose: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, workload, purpose, index])))


def ternary(n: int, seed: int = 0, workload: int = 0, index: int = 0) -> np.ndarray:
    """Uniform ternary vector (int8) of length n."""
    return rng(seed, workload, SECRET, index).integers(-1, 2, size=n, dtype=np.int64).astype(np.int8)


def ternary_hw(n: int, weight: int, seed: int = 0, workload: int = 0, index: int = 0) -> np.ndarray:
    """Ternary vector (int8) with exactly `weight` nonzero entries, each +1 or -1 uniformly,
    at uniformly chosen positions (the sparse secret of the paper's parameter section)."""
    g = rng(seed, workload, SECRET, index)
    pos = g.choice(n, size=weight, replace=False)
    s = np.zeros(n, dtype=np.int8)
    s[pos] = np.where(g.integers(0, 2, size=weight) == 1, 1, -1).astype(np.int8)
    return s


def gaussian(n: int, seed: int = 0, workload: int = 0, purpose: int = ERROR, index: int = 0) -> np.ndarray:
    """Rounded (half-even) clipped normal deviates, int32, sigma = 3.2."""
    x = rng(seed, workload, purpose, index).normal(0.0, SIGMA, size=n)
    return np.clip(np.rint(x), -ERROR_CLIP, ERROR_CLIP).astype(np.int32)


def uniform_residues(moduli, n: int, seed: int = 0, workload: int = 0, purpose: int = UNIFORM,
                     index: int = 0) -> np.ndarray:
    """Array [len(moduli)][n] of uint64, row i uniform in [0, moduli[i])."""
    g = rng(seed, workload, purpose, index)
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, q in enumerate(moduli):
        out[i] = g.integers(0, int(q), size=n, dtype=np.uint64)
    return out


def slot_values(count: int, bound: int, seed: int = 0, workload: int = 0, index: int = 0) -> np.ndarray:
    """Uniform integers in [0, bound), uint64."""
    return rng(seed, workload, SLOTS, index).integers(0, bound, size=count, dtype=np.uint64)


def int8_activations(count: int, sigma: float = 32.0, seed: int = 0, workload: int = 0,
                     index: int = 0) -> np.ndarray:
    """Signed activations: round-half-even of N(0, sigma^2), clipped to [-128, 127] (int64)."""
    x = rng(seed, workload, SLOTS, index).normal(0.0, sigma, size=count)
    return np.clip(np.rint(x), -128, 127).astype(np.int64)


def key_randomness(moduli, n: int, n_digits: int, seed: int = 0, workload: int = 0, key_index: int = 0):
    """Randomness for one switching key with n_digits digits.

    Returns (a, e): a is uint64 [n_digits][len(moduli)][n] with row i uniform mod
    moduli[i]; e is int32 [n_digits][n] from the clipped Gaussian.
    """
    a = np.empty((n_digits, len(moduli), n), dtype=np.uint64)
    e = np.empty((n_digits, n), dtype=np.int32)
    for j in range(n_digits):
        idx = key_index * 4096 + j
        a[j] = uniform_residues(moduli, n, seed, workload, KEY_A, idx)
        e[j] = gaussian(n, seed, workload, KEY_E, idx)
    return a, e


def encryption_randomness(moduli, n: int, seed: int = 0, workload: int = 0, index: int = 0):
    """(c1, e) for one fresh encryption: c1 uint64 [len(moduli)][n], e int32 [n]."""
    c1 = uniform_residues(moduli, n, seed, workload, ENC_C1, index)
    e = gaussian(n, seed, workload, ENC_E, index)
    return c1, e
