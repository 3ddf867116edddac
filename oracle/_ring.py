"""ctypes loader for the oracle's exact C kernels (ring.c).  Test infrastructure only."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libring.so")
_SRC = os.path.join(_HERE, "ring.c")


def build():
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _SO, _SRC])


def _load():
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_SO)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i64 = ctypes.c_int64
    u64 = ctypes.c_uint64
    lib.o_powmod.restype = u64
    lib.o_powmod.argtypes = [u64, u64, u64]
    lib.o_negacyclic_dot.argtypes = [u64p, u64p, i64, u64p, i64, u64]
    lib.o_negacyclic_dot_at.argtypes = [u64p, u64p, i64, i64p, i64, u64p, i64, u64]
    lib.o_negacyclic_mul_small.argtypes = [u64p, i64p, u64p, i64, u64]
    lib.o_mulmod_vec.argtypes = [u64p, u64p, u64p, i64, u64]
    lib.o_mulmod_scalar.argtypes = [u64p, u64, u64p, i64, u64]
    lib.o_ntt_def.argtypes = [u64p, u64p, i64, u64, u64]
    lib.o_intt_def.argtypes = [u64p, u64p, i64, u64, u64, u64p]
    lib.o_ntt_def_at.argtypes = [u64p, i64p, i64, u64p, i64, u64, u64]
    return lib


_lib = _load()


def _p(a, t=ctypes.c_uint64):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def negacyclic_dot(a, b, q):
    """sum_t a[t] * b[t] in Z_q[X]/(X^N+1); a, b of shape [T][N] (or [N])."""
    a = _u64(a)
    b = _u64(b)
    if a.ndim == 1:
        a = a[None]
        b = b[None]
    T, N = a.shape
    out = np.empty(N, dtype=np.uint64)
    _lib.o_negacyclic_dot(_p(a), _p(b), T, _p(out), N, int(q))
    return out


def negacyclic_dot_at(a, b, q, idx):
    a = _u64(a)
    b = _u64(b)
    if a.ndim == 1:
        a = a[None]
        b = b[None]
    T, N = a.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx), dtype=np.uint64)
    _lib.o_negacyclic_dot_at(_p(a), _p(b), T, _p(idx, ctypes.c_int64), len(idx), _p(out), N, int(q))
    return out


def negacyclic_mul_small(a, s, q):
    a = _u64(a)
    s = np.ascontiguousarray(s, dtype=np.int64)
    out = np.empty_like(a)
    _lib.o_negacyclic_mul_small(_p(a), _p(s, ctypes.c_int64), _p(out), a.shape[0], int(q))
    return out


def mulmod_vec(a, b, q):
    a = _u64(a)
    b = _u64(b)
    out = np.empty_like(a)
    _lib.o_mulmod_vec(_p(a), _p(b), _p(out), a.size, int(q))
    return out


def mulmod_scalar(a, s, q):
    a = _u64(a)
    out = np.empty_like(a)
    _lib.o_mulmod_scalar(_p(a), int(s) % int(q), _p(out), a.size, int(q))
    return out


def powmod(b, e, q):
    return int(_lib.o_powmod(int(b) % int(q), int(e), int(q)))


def ntt_def(a, q, psi):
    a = _u64(a)
    out = np.empty_like(a)
    _lib.o_ntt_def(_p(a), _p(out), a.shape[0], int(q), int(psi))
    return out


def intt_def(a, q, psi):
    a = _u64(a)
    out = np.empty_like(a)
    scratch = np.empty(2 * a.shape[0], dtype=np.uint64)
    _lib.o_intt_def(_p(a), _p(out), a.shape[0], int(q), int(psi), _p(scratch))
    return out


def ntt_def_at(a, q, psi, idx):
    a = _u64(a)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx), dtype=np.uint64)
    _lib.o_ntt_def_at(_p(a), _p(idx, ctypes.c_int64), len(idx), _p(out), a.shape[0], int(q), int(psi))
    return out
