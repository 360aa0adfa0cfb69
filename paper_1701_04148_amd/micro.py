"""ctypes binding of libsf_micro.so (include/sf_micro.h): the copy and
random-access kernels that give the ceilings the sketch is measured against."""
from __future__ import annotations

import ctypes
import os

from . import PKG

MICRO_PATH = os.path.join(PKG, "libsf_micro.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(MICRO_PATH):
            raise ImportError(f"{MICRO_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(MICRO_PATH)
        P, U64, U32, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.micro_copy.restype = I
        L.micro_copy.argtypes = [P, P, U64, P]
        for n in ("micro_gather_u32", "micro_gather_16b"):
            getattr(L, n).restype = I
            getattr(L, n).argtypes = [P, U64, U64, U32, P, P]
        L.micro_gather_pair.restype = I
        L.micro_gather_pair.argtypes = [P, U64, U64, U32, U32, P, P]
        L.micro_num_xcc.restype = I
        L.micro_num_xcc.argtypes = []
        L.micro_atomic_add_xcd.restype = I
        L.micro_atomic_add_xcd.argtypes = [P, U64, U64, U32, U32, U32, P]
        L.micro_atomic_add_u32.restype = I
        L.micro_atomic_add_u32.argtypes = [P, U64, U64, U32, P]
        L.micro_scatter_u64.restype = I
        L.micro_scatter_u64.argtypes = [P, U64, U64, U32, P]
        _lib = L
    return _lib


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream or None


def _ok(rc, what):
    if rc:
        raise RuntimeError(f"{what} failed ({rc})")


def copy(src, dst, nbytes: int):
    _ok(lib().micro_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream()), "micro_copy")


def gather_u32(table, n: int, seed: int, sink):
    _ok(lib().micro_gather_u32(table.data_ptr(), table.numel(), n, seed, sink.data_ptr(), _stream()),
        "micro_gather_u32")


def gather_16b(table, n: int, seed: int, sink):
    _ok(lib().micro_gather_16b(table.data_ptr(), table.numel(), n, seed, sink.data_ptr(), _stream()),
        "micro_gather_16b")


def atomic_add_u32(table, n: int, seed: int):
    _ok(lib().micro_atomic_add_u32(table.data_ptr(), table.numel(), n, seed, _stream()),
        "micro_atomic_add_u32")


def atomic_add_xcd(table, n: int, seed: int, nxcc: int, wg_scope: bool):
    _ok(lib().micro_atomic_add_xcd(table.data_ptr(), table.numel(), n, seed, nxcc, int(wg_scope),
                                   _stream()), "micro_atomic_add_xcd")


def num_xcc() -> int:
    return int(lib().micro_num_xcc())


def gather_pair(table, n: int, seed: int, same_line: bool, sink):
    _ok(lib().micro_gather_pair(table.data_ptr(), table.numel(), n, seed, int(same_line),
                                sink.data_ptr(), _stream()), "micro_gather_pair")


def scatter_u64(table, n: int, seed: int):
    _ok(lib().micro_scatter_u64(table.data_ptr(), table.numel(), n, seed, _stream()), "micro_scatter_u64")
