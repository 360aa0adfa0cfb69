"""SF-sketch CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain sequential implementation of the Slim-Fat sketch (arXiv:1701.04148,
Section 3.5, final version SF_F) used to check the HIP path.  Only the test
suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import it; the product package never does, and this module imports
nothing from the product package.

The arithmetic lives in ``sf_oracle.c`` (plain C, gcc -O2, single thread);
this module compiles it and marshals numpy arrays.  ``sfpy`` holds a second,
pure-Python transcription for tiny streams.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, EUNDERFLOW = 0, -1, -2, -5
SLIM_MAX = 65535


def build() -> str:
    """Compile the C oracle into liboracle.so (gcc, -O2, no SIMD intrinsics)."""
    src = os.path.join(_HERE, "sf_oracle.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, src])
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.oracle_murmur3_32.restype = U32
        L.oracle_murmur3_32.argtypes = [P, U64, U32]
        L.oracle_create.restype = P
        L.oracle_create.argtypes = [U32, U32, U32, U32, U32]
        L.oracle_destroy.argtypes = [P]
        L.oracle_get_state.argtypes = [P, P, P]
        L.oracle_set_state.argtypes = [P, P, P]
        L.oracle_indices.argtypes = [P, P, U64, P, P]
        for name in ("oracle_seq",):
            getattr(L, name).restype = I
            getattr(L, name).argtypes = [P, P, P, U64, I]
        L.oracle_seq_idx.restype = I
        L.oracle_seq_idx.argtypes = [P, P, P, P, U64, I]
        L.oracle_batch.restype = I
        L.oracle_batch.argtypes = [P, P, P, U64, U64, I]
        L.oracle_batch_idx.restype = I
        L.oracle_batch_idx.argtypes = [P, P, P, P, U64, U64, I]
        L.oracle_query.argtypes = [P, P, U64, P]
        L.oracle_query_idx.argtypes = [P, P, U64, P]
        L.oracle_fat_histogram.argtypes = [P, P, P, U64, P]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _key_bytes_array(keys: np.ndarray, key_bytes: int) -> np.ndarray:
    a = np.ascontiguousarray(keys)
    if key_bytes == 4 and a.dtype != np.uint8:
        a = np.ascontiguousarray(a.astype("<u4", copy=False))
    if a.nbytes % key_bytes:
        raise ValueError("key array size is not a multiple of key_bytes")
    return a


def murmur3_32(data: bytes, seed: int) -> int:
    buf = np.frombuffer(bytes(data), dtype=np.uint8) if data else np.zeros(1, np.uint8)
    return int(lib().oracle_murmur3_32(buf.ctypes.data, len(data), seed & 0xFFFFFFFF))


class Sketch:
    """Oracle SF_F sketch: Fat uint32 [d][w][z], Slim uint16 [d][w]."""

    def __init__(self, d: int, w: int, z: int, key_bytes: int = 4, seed_base: int = 1):
        self.d, self.w, self.z, self.key_bytes, self.seed_base = d, w, z, key_bytes, seed_base
        self._h = lib().oracle_create(d, w, z, key_bytes, seed_base)
        if not self._h:
            raise ValueError("invalid oracle sketch shape")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    # -- state
    def fat(self) -> np.ndarray:
        out = np.empty((self.d, self.w, self.z), dtype=np.uint32)
        lib().oracle_get_state(self._h, out.ctypes.data, None)
        return out

    def slim(self) -> np.ndarray:
        out = np.empty((self.d, self.w), dtype=np.uint16)
        lib().oracle_get_state(self._h, None, out.ctypes.data)
        return out

    def set_state(self, fat=None, slim=None):
        fat = None if fat is None else np.ascontiguousarray(fat, dtype=np.uint32)
        slim = None if slim is None else np.ascontiguousarray(slim, dtype=np.uint16)
        lib().oracle_set_state(self._h, _ptr(fat), _ptr(slim))

    def indices(self, keys: np.ndarray):
        kb = _key_bytes_array(keys, self.key_bytes)
        n = kb.nbytes // self.key_bytes
        h = np.empty((n, self.d), dtype=np.uint32)
        f = np.empty((n, self.d), dtype=np.uint32)
        lib().oracle_indices(self._h, kb.ctypes.data, n, h.ctypes.data, f.ctypes.data)
        return h, f

    # -- updates
    def _ops(self, ops, n):
        if ops is None:
            return None
        o = np.ascontiguousarray(ops, dtype=np.uint8)
        if o.size != n:
            raise ValueError("ops length mismatch")
        return o

    def seq(self, keys, ops=None, checked=False) -> int:
        kb = _key_bytes_array(keys, self.key_bytes)
        n = kb.nbytes // self.key_bytes
        o = self._ops(ops, n)
        return lib().oracle_seq(self._h, kb.ctypes.data, _ptr(o), n, int(checked))

    def batch(self, keys, ops=None, b=1, checked=False) -> int:
        kb = _key_bytes_array(keys, self.key_bytes)
        n = kb.nbytes // self.key_bytes
        o = self._ops(ops, n)
        return lib().oracle_batch(self._h, kb.ctypes.data, _ptr(o), n, int(b), int(checked))

    def seq_idx(self, h, f, ops=None, checked=False) -> int:
        h = np.ascontiguousarray(h, dtype=np.uint32)
        f = np.ascontiguousarray(f, dtype=np.uint32)
        n = h.shape[0]
        o = self._ops(ops, n)
        return lib().oracle_seq_idx(self._h, h.ctypes.data, f.ctypes.data, _ptr(o), n, int(checked))

    def batch_idx(self, h, f, ops=None, b=1, checked=False) -> int:
        h = np.ascontiguousarray(h, dtype=np.uint32)
        f = np.ascontiguousarray(f, dtype=np.uint32)
        n = h.shape[0]
        o = self._ops(ops, n)
        return lib().oracle_batch_idx(self._h, h.ctypes.data, f.ctypes.data, _ptr(o), n, int(b),
                                      int(checked))

    # -- queries
    def query(self, keys) -> np.ndarray:
        kb = _key_bytes_array(keys, self.key_bytes)
        n = kb.nbytes // self.key_bytes
        out = np.empty(n, dtype=np.uint32)
        lib().oracle_query(self._h, kb.ctypes.data, n, out.ctypes.data)
        return out

    def query_idx(self, h) -> np.ndarray:
        h = np.ascontiguousarray(h, dtype=np.uint32)
        out = np.empty(h.shape[0], dtype=np.uint32)
        lib().oracle_query_idx(self._h, h.ctypes.data, h.shape[0], out.ctypes.data)
        return out

    def fat_histogram(self, keys, ops=None) -> np.ndarray:
        kb = _key_bytes_array(keys, self.key_bytes)
        n = kb.nbytes // self.key_bytes
        o = self._ops(ops, n)
        out = np.zeros((self.d, self.w, self.z), dtype=np.uint32)
        lib().oracle_fat_histogram(self._h, kb.ctypes.data, _ptr(o), n, out.ctypes.data)
        return out


def query_slim(slim: np.ndarray, d: int, w: int, z: int, keys, key_bytes: int = 4,
               seed_base: int = 1) -> np.ndarray:
    """Collector-side query over an exported Slim (Section 3.1 query rule)."""
    sk = Sketch(d, w, z, key_bytes, seed_base)
    sk.set_state(slim=slim)
    return sk.query(keys)
