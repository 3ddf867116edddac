"""Thin ctypes binding of libbgv.so (include/bgv.h).

Argument marshalling only: every step of the arithmetic runs in the library's
gfx950 kernels.  PyTorch provides device memory (uint64 words stored in int64
tensors) and the stream.  If the shared library is missing this module raises
at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbgv.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")
_lib = ctypes.CDLL(LIB_PATH)

ROW_SWAP = -1
NOALLOC_SCRATCH_WORDS = 4 * 1024 * 1024  # BGV_NOALLOC_SCRATCH_WORDS
OP_LT = 0
OP_EQ = 1
OP_GT = 2
OP_LE = 3
OP_GE = 4
OP_NEQ = 5

STATUS = {0: "OK", 1: "E_ARG", 2: "E_PARAM", 3: "E_LEVEL", 4: "E_PTXT_MOD", 5: "E_NOKEY", 6: "E_OOM",
          7: "E_DEVICE", 8: "E_UNSUPPORTED"}


class BgvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_int32), ("p", ctypes.c_int32), ("r", ctypes.c_int32), ("L", ctypes.c_int32),
                ("K", ctypes.c_int32)]


class _Ct(ctypes.Structure):
    _fields_ = [("d", ctypes.c_void_p), ("cap_words", ctypes.c_int64), ("n", ctypes.c_int32),
                ("level", ctypes.c_int32), ("t_exp", ctypes.c_int32), ("noise", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("N", "log_n", "p", "r", "L", "K", "alpha", "dnum", "slots", "d")] + \
               [("t", ctypes.c_int64), ("max_batch", ctypes.c_int32), ("_pad", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("key_switches", "rescale_drops", "limb_drops", "odd_splits",
                                              "algo_bytes")] + \
               [(f, ctypes.c_int32) for f in ("max_baby_k", "max_inner_terms", "max_inner_outputs",
                                              "max_tensor_pairs")]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_P = ctypes.POINTER
_sigs = {
    "bgv_ctx_create": [_P(_Params), _vp, _P(_vp)],
    "bgv_ctx_destroy": [_vp],
    "bgv_set_stream": [_vp, _vp],
    "bgv_ctx_info": [_vp, _P(_Info)],
    "bgv_ctx_primes": [_vp, _vp],
    "bgv_ct_words": [_vp, _i32],
    "bgv_sync": [_vp],
    "bgv_last_error": [_vp],
    "bgv_keygen": [_vp, _vp, _vp, _vp, _vp, _i32, _i32, _P(_vp)],
    "bgv_keys_destroy": [_vp],
    "bgv_keys_bytes": [_vp],
    "bgv_encrypt": [_vp, _vp, _vp, _vp, _vp, _P(_Ct)],
    "bgv_decrypt": [_vp, _vp, _P(_Ct), _vp, _vp],
    "bgv_add": [_vp, _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_sub": [_vp, _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_negate": [_vp, _P(_Ct), _P(_Ct)],
    "bgv_mul_scalar": [_vp, _P(_Ct), _i64, _P(_Ct)],
    "bgv_add_const": [_vp, _P(_Ct), _i64, _P(_Ct)],
    "bgv_divide_by_p": [_vp, _P(_Ct), _P(_Ct)],
    "bgv_set_t_exp": [_vp, _P(_Ct), _i32],
    "bgv_mul_relin": [_vp, _vp, _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_rotate": [_vp, _vp, _P(_Ct), _i32, _P(_Ct)],
    "bgv_mod_switch": [_vp, _P(_Ct), _P(_Ct)],
    "bgv_mod_switch_to": [_vp, _P(_Ct), _i32, _P(_Ct)],
    "bgv_eval_poly": [_vp, _vp, _P(_Ct), _vp, _i32, _P(_Ct)],
    "bgv_space_reduce": [_vp, _vp, _P(_Ct), _P(_Ct)],
    "bgv_compare": [_vp, _vp, _P(_Ct), _i32, _i32, _P(_Ct)],
    "bgv_space_raise": [_vp, _vp, _P(_Ct), _P(_Ct)],
    "bgv_less_than": [_vp, _vp, _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_rotate_sum": [_vp, _vp, _P(_Ct), _P(_Ct)],
    "bgv_mul": [_vp, _vp, _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_batch_sum": [_vp, _P(_Ct), _P(_Ct)],
    "bgv_filter_sum": [_vp, _vp, _P(_Ct), _P(_Ct), _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_relu": [_vp, _vp, _P(_Ct), _P(_Ct)],
    "bgv_filter_products": [_vp, _vp, _P(_Ct), _P(_Ct), _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_ntt": [_vp, _vp, _i64, _i32, _i32, _i32],
    "bgv_set_ntt_chunk": [_vp, _i32],
    "bgv_trim": [_vp, _vp],
    "bgv_set_ntt_split": [_vp, _i32],
    "bgv_set_schedule": [_vp, _i32],
    "bgv_autotune_ntt": [_vp, _i32, _i32, _vp, _vp],
    "bgv_capture_begin": [_vp],
    "bgv_capture_end": [_vp, _P(_vp)],
    "bgv_graph_launch": [_vp, _vp],
    "bgv_graph_destroy": [_vp],
    "bgv_get_ntt_chunk": [_vp],
    "bgv_get_stats": [_vp, _P(_Stats)],
    "bgv_mod_switch_noalloc": [_vp, _P(_Ct), _P(_Ct)],
    "bgv_set_ntt_coop": [_vp, _i32, _i32],
    "bgv_set_modup_fused": [_vp, _i32],
    "bgv_set_moddown_fused": [_vp, _i32],
    "bgv_filter_and_products": [_vp, _vp, _i32, _vp, _vp, _vp, _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_filter_and_sum": [_vp, _vp, _i32, _vp, _vp, _vp, _P(_Ct), _P(_Ct), _P(_Ct)],
    "bgv_reset_stats": [_vp],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.bgv_ctx_destroy.restype = None
_lib.bgv_keys_destroy.restype = None
_lib.bgv_graph_destroy.restype = None
_lib.bgv_last_error.restype = ctypes.c_char_p
_lib.bgv_ct_words.restype = ctypes.c_int64
_lib.bgv_keys_bytes.restype = ctypes.c_int64

EXPORTED = tuple(_sigs)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Ct:
    """A batch of n ciphertexts in a device tensor (int64 words holding uint64 residues).

    noise: the library's noise estimate of the batch (sixteenths of a bit, 0 = unknown)."""

    def __init__(self, tensor: torch.Tensor, n: int, level: int, t_exp: int, noise: int = 0):
        self.tensor = tensor
        self.n, self.level, self.t_exp, self.noise = n, level, t_exp, noise

    def _struct(self) -> _Ct:
        return _Ct(self.tensor.data_ptr(), self.tensor.numel(), self.n, self.level, self.t_exp, self.noise)

    def _update(self, s: _Ct):
        self.n, self.level, self.t_exp, self.noise = s.n, s.level, s.t_exp, s.noise

    def words(self, N: int) -> np.ndarray:
        """uint64 array [n][2][level][N] copied to the host."""
        used = self.n * 2 * self.level * N
        return self.tensor[:used].cpu().numpy().view(np.uint64).reshape(self.n, 2, self.level, N)


class Keys:
    def __init__(self, ctx: "Context", handle: ctypes.c_void_p):
        self._ctx = ctx
        self.handle = handle

    @property
    def bytes(self) -> int:
        return int(_lib.bgv_keys_bytes(self.handle))

    def __del__(self, _destroy=_lib.bgv_keys_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


class Graph:
    """A captured sequence of library operations, replayed with the same buffers."""

    def __init__(self, ctx: "Context", handle: ctypes.c_void_p):
        self._ctx = ctx
        self.handle = handle

    def launch(self):
        self._ctx._check(_lib.bgv_graph_launch(self._ctx.handle, self.handle))

    def __del__(self, _destroy=_lib.bgv_graph_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


class Context:
    def __init__(self, log_n: int, p: int, r: int, L: int, K: int, device: str = "cuda:0", stream=None):
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        prm = _Params(log_n, p, r, L, K)
        st = _lib.bgv_ctx_create(ctypes.byref(prm), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        self.handle = h
        if st != 0:
            msg = _lib.bgv_last_error(h).decode() if h else ""
            _lib.bgv_ctx_destroy(h)
            self.handle = None
            raise BgvError(st, msg)
        info = _Info()
        _lib.bgv_ctx_info(h, ctypes.byref(info))
        self.N, self.log_n, self.p, self.r = info.N, info.log_n, info.p, info.r
        self.L, self.K, self.alpha, self.dnum = info.L, info.K, info.alpha, info.dnum
        self.slots, self.d, self.t = info.slots, info.d, info.t
        self.max_batch = info.max_batch
        pr = np.empty(L + K, dtype=np.uint64)
        _lib.bgv_ctx_primes(h, _ptr(pr))
        self.primes = [int(x) for x in pr]

    def __del__(self, _destroy=_lib.bgv_ctx_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None

    # ------------------------------------------------------------------ helpers
    def _check(self, st):
        if st != 0:
            raise BgvError(st, _lib.bgv_last_error(self.handle).decode())

    def words(self, level: int) -> int:
        return int(_lib.bgv_ct_words(self.handle, level))

    def empty(self, n: int, level: int, t_exp: int = None) -> Ct:
        t = torch.empty(n * self.words(level), dtype=torch.int64, device=self.device)
        return Ct(t, n, level, self.r if t_exp is None else t_exp)

    def from_words(self, words: np.ndarray, t_exp: int) -> Ct:
        """Upload uint64 words [n][2][level][N] (evaluation form) as a batch."""
        w = np.ascontiguousarray(words, dtype=np.uint64)
        n, _, level, _ = w.shape
        t = torch.from_numpy(w.reshape(-1).view(np.int64)).to(self.device)
        return Ct(t, n, level, t_exp)

    def view(self, ct: Ct, start: int, count: int) -> Ct:
        """Ciphertexts start .. start+count-1 of a batch, sharing its memory."""
        per = self.words(ct.level)
        return Ct(ct.tensor[start * per:(start + count) * per], count, ct.level, ct.t_exp, ct.noise)

    def concat(self, parts, out: Ct = None) -> Ct:
        """Copy batches of equal level and t_exp into one contiguous batch."""
        n = sum(p.n for p in parts)
        lv, te = parts[0].level, parts[0].t_exp
        out = out or self.empty(n, lv, te)
        per = self.words(lv)
        pos = 0
        for p in parts:
            assert p.level == lv and p.t_exp == te
            out.tensor[pos * per:(pos + p.n) * per].copy_(p.tensor[:p.n * per])
            pos += p.n
        out.n, out.level, out.t_exp = n, lv, te
        # the largest estimate bounds every part (unknown if any part is)
        out.noise = 0 if any(p.noise <= 0 for p in parts) else max(p.noise for p in parts)
        return out

    def sync(self):
        self._check(_lib.bgv_sync(self.handle))

    def capture_begin(self):
        self._check(_lib.bgv_capture_begin(self.handle))

    def capture_end(self) -> Graph:
        h = ctypes.c_void_p()
        self._check(_lib.bgv_capture_end(self.handle, ctypes.byref(h)))
        return Graph(self, h)

    def set_moddown_fused(self, mode: int):
        """The product step's ModDown and switch fused with the passes around them: 0 never, 1 (the default)
        when the batch is large enough for the fused kernel to pay, 2 always."""
        self._check(_lib.bgv_set_moddown_fused(self.handle, int(mode)))

    def set_modup_fused(self, on: bool):
        """Key switching with the fused ModUp pass (True, the default) or ModUp between full transforms."""
        self._check(_lib.bgv_set_modup_fused(self.handle, 1 if on else 0))

    def set_ntt_coop(self, mode: int, lookahead: int = 2):
        """Two-pass transforms as one XCD-local launch (mode 1) or two launches (mode 0)."""
        self._check(_lib.bgv_set_ntt_coop(self.handle, int(mode), int(lookahead)))

    def stats(self) -> dict:
        """Host-side counters of the enqueued work (see bgv_get_stats)."""
        st = _Stats()
        self._check(_lib.bgv_get_stats(self.handle, ctypes.byref(st)))
        return {f: int(getattr(st, f)) for f, _ in _Stats._fields_}

    def reset_stats(self):
        self._check(_lib.bgv_reset_stats(self.handle))

    def trim(self) -> int:
        """Free the library's cached scratch; returns the bytes still in use."""
        held = ctypes.c_int64()
        self._check(_lib.bgv_trim(self.handle, ctypes.byref(held)))
        return held.value

    # ------------------------------------------------------------------ keys and encryption
    def keygen(self, s, a, e, steps=(), with_conj=False) -> Keys:
        s = np.ascontiguousarray(s, dtype=np.int8)
        a = np.ascontiguousarray(a, dtype=np.uint64)
        e = np.ascontiguousarray(e, dtype=np.int32)
        st_arr = np.ascontiguousarray(list(steps) or [0], dtype=np.int32)
        h = ctypes.c_void_p()
        self._check(_lib.bgv_keygen(self.handle, _ptr(s), _ptr(a), _ptr(e), _ptr(st_arr), len(steps),
                                    1 if with_conj else 0, ctypes.byref(h)))
        return Keys(self, h)

    def encrypt(self, s, slots, c1, e, out: Ct = None) -> Ct:
        slots = np.ascontiguousarray(slots, dtype=np.uint64).reshape(-1, self.slots)
        n = slots.shape[0]
        s = np.ascontiguousarray(s, dtype=np.int8)
        c1 = np.ascontiguousarray(c1, dtype=np.uint64).reshape(n, self.L, self.N)
        e = np.ascontiguousarray(e, dtype=np.int32).reshape(n, self.N)
        out = out or self.empty(n, self.L)
        out.n = n
        cs = out._struct()
        self._check(_lib.bgv_encrypt(self.handle, _ptr(s), _ptr(slots), _ptr(c1), _ptr(e), ctypes.byref(cs)))
        out._update(cs)
        return out

    def decrypt(self, s, ct: Ct, with_flags: bool = False):
        s = np.ascontiguousarray(s, dtype=np.int8)
        slots = np.empty(ct.n * self.slots, dtype=np.uint64)
        flags = np.empty(ct.n * self.slots, dtype=np.uint8) if with_flags else None
        cs = ct._struct()
        self._check(_lib.bgv_decrypt(self.handle, _ptr(s), ctypes.byref(cs), _ptr(slots),
                                     _ptr(flags) if with_flags else None))
        slots = slots.reshape(ct.n, self.slots)
        return (slots, flags.reshape(ct.n, self.slots)) if with_flags else slots

    # ------------------------------------------------------------------ operations
    def _out(self, out, n, level, t_exp):
        return out if out is not None else self.empty(n, level, t_exp)

    def _bin(self, fn, a: Ct, b: Ct, out: Ct = None, keys: Keys = None) -> Ct:
        out = self._out(out, a.n, a.level, a.t_exp)
        sa, sb, so = a._struct(), b._struct(), out._struct()
        if keys is None:
            self._check(fn(self.handle, ctypes.byref(sa), ctypes.byref(sb), ctypes.byref(so)))
        else:
            self._check(fn(self.handle, keys.handle, ctypes.byref(sa), ctypes.byref(sb), ctypes.byref(so)))
        out._update(so)
        return out

    def add(self, a, b, out=None):
        return self._bin(_lib.bgv_add, a, b, out)

    def sub(self, a, b, out=None):
        return self._bin(_lib.bgv_sub, a, b, out)

    def mul_relin(self, keys, a, b, out=None):
        return self._bin(_lib.bgv_mul_relin, a, b, out, keys)

    def _un(self, fn, a: Ct, *args, out: Ct = None, level=None, t_exp=None, keys=None) -> Ct:
        out = self._out(out, a.n, a.level if level is None else level, a.t_exp if t_exp is None else t_exp)
        sa, so = a._struct(), out._struct()
        if keys is None:
            self._check(fn(self.handle, ctypes.byref(sa), *args, ctypes.byref(so)))
        else:
            self._check(fn(self.handle, keys.handle, ctypes.byref(sa), *args, ctypes.byref(so)))
        out._update(so)
        return out

    def negate(self, a, out=None):
        return self._un(_lib.bgv_negate, a, out=out)

    def mul_scalar(self, a, c: int, out=None):
        return self._un(_lib.bgv_mul_scalar, a, ctypes.c_int64(int(c)), out=out)

    def add_const(self, a, c: int, out=None):
        return self._un(_lib.bgv_add_const, a, ctypes.c_int64(int(c)), out=out)

    def divide_by_p(self, a, out=None):
        return self._un(_lib.bgv_divide_by_p, a, out=out, t_exp=a.t_exp - 1)

    def set_t_exp(self, a: Ct, t_exp: int) -> Ct:
        s = a._struct()
        self._check(_lib.bgv_set_t_exp(self.handle, ctypes.byref(s), t_exp))
        return Ct(a.tensor, a.n, a.level, t_exp, a.noise)

    def rotate(self, keys, a, step: int, out=None):
        return self._un(_lib.bgv_rotate, a, ctypes.c_int32(step), out=out, keys=keys)

    def mod_switch(self, a, out=None):
        return self._un(_lib.bgv_mod_switch, a, out=out, level=a.level - 1)

    def mod_switch_noalloc(self, a, out):
        """bgv_mod_switch_noalloc: the single switch with the library's fixed scratch (no device
        allocation in the call); the caller provides the output batch."""
        sa, so = a._struct(), out._struct()
        self._check(_lib.bgv_mod_switch_noalloc(self.handle, ctypes.byref(sa), ctypes.byref(so)))
        out._update(so)
        return out

    def mod_switch_to(self, a, level: int, out=None):
        return self._un(_lib.bgv_mod_switch_to, a, ctypes.c_int32(level), out=out, level=level)

    def eval_poly(self, keys, a, coeffs, out=None):
        cf = np.ascontiguousarray([int(c) for c in coeffs], dtype=np.int64)
        out = self._out(out, a.n, a.level, a.t_exp)
        sa, so = a._struct(), out._struct()
        self._check(_lib.bgv_eval_poly(self.handle, keys.handle, ctypes.byref(sa), _ptr(cf), len(cf) - 1,
                                       ctypes.byref(so)))
        out._update(so)
        return out

    def space_reduce(self, keys, a, outs=None):
        outs = outs or [self.empty(a.n, a.level, 1) for _ in range(a.t_exp)]
        arr = (_Ct * len(outs))(*[o._struct() for o in outs])
        sa = a._struct()
        self._check(_lib.bgv_space_reduce(self.handle, keys.handle, ctypes.byref(sa), arr))
        for o, s in zip(outs, arr):
            o._update(s)
        return outs

    def compare(self, keys, digits, op=OP_LT, out=None):
        out = self._out(out, digits[0].n, digits[0].level, self.r)
        arr = (_Ct * len(digits))(*[d._struct() for d in digits])
        so = out._struct()
        self._check(_lib.bgv_compare(self.handle, keys.handle, arr, len(digits), op, ctypes.byref(so)))
        out._update(so)
        return out

    def space_raise(self, keys, a, out=None):
        return self._un(_lib.bgv_space_raise, a, out=out, keys=keys)

    def less_than(self, keys, x, y=None, out=None):
        out = self._out(out, x.n, x.level, x.t_exp)
        sx, so = x._struct(), out._struct()
        sy = y._struct() if y is not None else None
        self._check(_lib.bgv_less_than(self.handle, keys.handle, ctypes.byref(sx),
                                       ctypes.byref(sy) if sy is not None else None, ctypes.byref(so)))
        out._update(so)
        return out

    def rotate_sum(self, keys, a, out=None):
        return self._un(_lib.bgv_rotate_sum, a, out=out, keys=keys)

    def mul(self, keys, a, b, out=None):
        n = max(a.n, b.n)
        out = self._out(out, n, min(a.level, b.level) - 1, a.t_exp)
        sa, sb, so = a._struct(), b._struct(), out._struct()
        self._check(_lib.bgv_mul(self.handle, keys.handle, ctypes.byref(sa), ctypes.byref(sb), ctypes.byref(so)))
        out._update(so)
        return out

    def batch_sum(self, a, out=None):
        return self._un(_lib.bgv_batch_sum, a, out=out) if out is not None else self._un(
            _lib.bgv_batch_sum, a, out=self.empty(1, a.level, a.t_exp))

    def filter_sum(self, keys, a, thr, b, c, out=None):
        out = self._out(out, 1, a.level, a.t_exp)
        s = [x._struct() for x in (a, thr, b, c, out)]
        self._check(_lib.bgv_filter_sum(self.handle, keys.handle, *[ctypes.byref(x) for x in s]))
        out._update(s[-1])
        return out

    def filter_products(self, keys, a, thr, b, c, out=None):
        out = self._out(out, a.n, a.level, a.t_exp)
        s = [x._struct() for x in (a, thr, b, c, out)]
        self._check(_lib.bgv_filter_products(self.handle, keys.handle, *[ctypes.byref(x) for x in s]))
        out._update(s[-1])
        return out

    def _filter_and(self, fn, keys, preds, b, c, out):
        """preds: list of (column batch, threshold ciphertext or batch, op code)."""
        cols = (_Ct * len(preds))(*[p[0]._struct() for p in preds])
        thrs = (_Ct * len(preds))(*[p[1]._struct() for p in preds])
        ops = np.ascontiguousarray([int(p[2]) for p in preds], dtype=np.int32)
        sb, sc, so = b._struct(), c._struct(), out._struct()
        self._check(fn(self.handle, keys.handle, len(preds), ctypes.cast(cols, _vp), ctypes.cast(thrs, _vp),
                       _ptr(ops), ctypes.byref(sb), ctypes.byref(sc), ctypes.byref(so)))
        out._update(so)
        return out

    def filter_and_products(self, keys, preds, b, c, out=None):
        return self._filter_and(_lib.bgv_filter_and_products, keys, preds, b, c,
                                self._out(out, b.n, b.level, b.t_exp))

    def filter_and_sum(self, keys, preds, b, c, out=None):
        return self._filter_and(_lib.bgv_filter_and_sum, keys, preds, b, c, self._out(out, 1, b.level, b.t_exp))

    def relu(self, keys, x, out=None):
        return self._un(_lib.bgv_relu, x, out=out, keys=keys)

    def set_ntt_split(self, first_pass_stages: int):
        self._check(_lib.bgv_set_ntt_split(self.handle, int(first_pass_stages)))

    SCHEDULES = {"fast": 0, "basic": 1}

    def set_schedule(self, name: str):
        """Polynomial evaluation schedule of the context: "fast" (default) or "basic"."""
        self._check(_lib.bgv_set_schedule(self.handle, self.SCHEDULES[name]))

    def autotune_ntt(self, limbs: int, reps: int = 10):
        """Pick the fastest NTT pass split for `limbs` limbs; returns (split, microseconds)."""
        s = ctypes.c_int32()
        us = ctypes.c_float()
        self._check(_lib.bgv_autotune_ntt(self.handle, int(limbs), int(reps), ctypes.byref(s), ctypes.byref(us)))
        return s.value, us.value

    @property
    def ntt_chunk(self) -> int:
        return int(_lib.bgv_get_ntt_chunk(self.handle))

    @ntt_chunk.setter
    def ntt_chunk(self, limbs: int):
        self._check(_lib.bgv_set_ntt_chunk(self.handle, int(limbs)))

    def ntt(self, t: torch.Tensor, n_polys: int, level: int, inverse: bool = False):
        self._check(_lib.bgv_ntt(self.handle, ctypes.c_void_p(t.data_ptr()), t.numel(), n_polys, level,
                                 1 if inverse else 0))
        return t
