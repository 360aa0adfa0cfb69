"""Python binding of libsf.so, the MI355X SF-sketch hot path (see include/sf.h).

Argument marshalling only: every step of insert, delete, query and export
runs in the library's HIP kernels.  PyTorch supplies device memory and the
HIP stream.  Importing this module does not need a GPU; the first call loads
libsf.so and raises if it has not been built (there is no CPU fallback).

Functions keep the C names (``sf_create``, ``sf_insert`` ...); ``Sketch``
wraps them for convenience.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsf.so")

SF_OK, SF_EINVAL, SF_ENOMEM, SF_EDEVICE, SF_ESTATE, SF_EUNDERFLOW = 0, -1, -2, -3, -4, -5
SLIM_MAX = 65535
NOALLOC_QUERY_COUNTERS = 1 << 23  # SF_NOALLOC_QUERY_COUNTERS of sf.h

_lib = None


class SFError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {sf_strerror(status)} ({status}){': ' + detail if detail else ''}")


class sf_config(ctypes.Structure):
    _fields_ = [("d", ctypes.c_uint32), ("w", ctypes.c_uint32), ("z", ctypes.c_uint32),
                ("key_bytes", ctypes.c_uint32), ("seed_base", ctypes.c_uint32),
                ("batch_ops", ctypes.c_uint32)]


KERNEL_KINDS = ("snapshot", "fat_add", "raise", "fat_sub", "clamp", "query", "export", "merge",
                "partition", "pairs", "own_step", "level", "own_final")
SF_K_COUNT = 16


class sf_kernel_stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * SF_K_COUNT), ("launches", ctypes.c_uint64 * SF_K_COUNT),
                ("items", ctypes.c_uint64 * SF_K_COUNT)]


# (name, restype, argtypes) of every entry point declared in include/sf.h
_P, _U64, _I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
_CFG = ctypes.POINTER(sf_config)
SIGNATURES = {
    "sf_footprint": (_U64, [_CFG]),
    "sf_create": (_I, [_CFG, _U64, _P, ctypes.POINTER(_P)]),
    "sf_destroy": (_I, [_P]),
    "sf_reset": (_I, [_P]),
    "sf_set_stream": (_I, [_P, _P]),
    "sf_insert": (_I, [_P, _P, _U64]),
    "sf_delete": (_I, [_P, _P, _U64]),
    "sf_update": (_I, [_P, _P, _P, _U64]),
    "sf_query": (_I, [_P, _P, _U64, _P]),
    "sf_query_slim": (_I, [_P, _CFG, _P, _U64, _P, _P]),
    "sf_query_host": (_I, [_P, _P, _U64, _P, ctypes.c_uint32]),
    "sf_query_slim_noalloc": (_I, [_P, _CFG, _P, _U64, _P, _P]),
    "sf_export_slim": (_I, [_P, _P, _U64]),
    "sf_export_fat": (_I, [_P, _P, _U64]),
    "sf_sync": (_I, [_P]),
    "sf_set_tile": (_I, [_P, ctypes.c_uint32]),
    "sf_set_merge": (_I, [_P, _I]),
    "sf_merge_path": (_I, [_P]),
    "sf_set_streams": (_I, [_P, _I]),
    "sf_set_owner_range": (_I, [_P, ctypes.c_uint32]),
    "sf_owner_range": (_I, [_P]),
    "sf_update_host": (_I, [_P, _P, _P, _U64, _U64]),
    "sf_merge_stats": (_I, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "sf_profile": (_I, [_P, _I]),
    "sf_profile_read": (_I, [_P, ctypes.POINTER(sf_kernel_stats), _I]),
    "sf_group_footprint": (_U64, [ctypes.c_uint32, _CFG, _U64]),
    "sf_group_create": (_I, [ctypes.c_uint32, _CFG, _U64, _U64, _P, ctypes.POINTER(_P)]),
    "sf_group_destroy": (_I, [_P]),
    "sf_group_reset": (_I, [_P]),
    "sf_group_insert": (_I, [_P, _P, _P]),
    "sf_group_delete": (_I, [_P, _P, _P]),
    "sf_group_update": (_I, [_P, _P, _P, _P]),
    "sf_group_query": (_I, [_P, _P, _P, _P]),
    "sf_group_export_slim": (_I, [_P, ctypes.c_uint32, _P, _U64]),
    "sf_group_export_fat": (_I, [_P, ctypes.c_uint32, _P, _U64]),
    "sf_group_sync": (_I, [_P]),
    "sf_group_set_graph": (_I, [_P, _I]),
    "sf_group_set_tile": (_I, [_P, ctypes.c_uint32]),
    "sf_group_set_merge": (_I, [_P, _I]),
    "sf_group_merge_path": (_I, [_P]),
    "sf_group_set_owner_ratio": (_I, [_P, ctypes.c_double]),
    "sf_group_merge_stats": (_I, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "sf_group_rounds": (_I, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "sf_group_profile": (_I, [_P, _I]),
    "sf_group_profile_read": (_I, [_P, ctypes.POINTER(sf_kernel_stats), _I]),
    "sf_pool_slot_bytes": (_U64, [_CFG]),
    "sf_pool_create": (_I, [_CFG, ctypes.c_uint32, _U64, _U64, _P, ctypes.POINTER(_P)]),
    "sf_pool_destroy": (_I, [_P]),
    "sf_pool_capacity": (_I, [_P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
    "sf_pool_acquire": (_I, [_P, ctypes.POINTER(ctypes.c_uint32)]),
    "sf_pool_release": (_I, [_P, ctypes.c_uint32]),
    "sf_pool_launch": (_I, [_P, _P, ctypes.c_uint32, ctypes.POINTER(_U64)]),
    "sf_pool_done": (_I, [_P, _U64]),
    "sf_pool_wait": (_I, [_P, _U64]),
    "sf_pool_export_slim": (_I, [_P, ctypes.c_uint32, _P, _U64, _I]),
    "sf_pool_export_fat": (_I, [_P, ctypes.c_uint32, _P, _U64]),
    "sf_pool_sync": (_I, [_P]),
    "sf_pool_set_tile": (_I, [_P, ctypes.c_uint32]),
    "sf_pool_set_merge": (_I, [_P, _I]),
    "sf_pool_set_owner_ratio": (_I, [_P, ctypes.c_double]),
    "sf_pool_merge_stats": (_I, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "sf_strerror": (ctypes.c_char_p, [_I]),
    "sf_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libsf.so; raise loudly when it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _lib = L
    return _lib


def sf_strerror(status: int) -> str:
    return lib().sf_strerror(status).decode()


def sf_last_error() -> str:
    return lib().sf_last_error().decode()


def _check(rc: int, where: str):
    if rc != SF_OK:
        raise SFError(rc, where, sf_last_error())


def _stream_handle(stream) -> int | None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _keys_ptr(keys, key_bytes: int):
    """(device pointer, n) of a contiguous GPU key tensor."""
    import torch
    if not isinstance(keys, torch.Tensor) or not keys.is_cuda:
        raise TypeError("keys must be a GPU tensor")
    if not keys.is_contiguous():
        raise ValueError("keys must be contiguous")
    nbytes = keys.numel() * keys.element_size()
    if key_bytes == 4:
        if keys.element_size() != 4:
            raise TypeError("uint32 keys need a 4-byte dtype (torch.int32 / torch.uint32)")
    elif keys.dtype != torch.uint8 or nbytes % 13:
        raise TypeError("13-byte keys need a uint8 tensor of n*13 bytes")
    return keys.data_ptr(), nbytes // key_bytes


def make_config(d: int, w: int, z: int, key_bytes: int = 4, seed_base: int = 1,
                batch_ops: int = 1 << 20) -> sf_config:
    return sf_config(d, w, z, key_bytes, seed_base, batch_ops)


def sf_footprint(cfg: sf_config) -> int:
    return int(lib().sf_footprint(ctypes.byref(cfg)))


def sf_create(cfg: sf_config, hbm_budget_bytes: int = 0, stream=None):
    h = ctypes.c_void_p()
    _check(lib().sf_create(ctypes.byref(cfg), hbm_budget_bytes, _stream_handle(stream),
                           ctypes.byref(h)), "sf_create")
    return h


def sf_destroy(h):
    _check(lib().sf_destroy(h), "sf_destroy")


def sf_reset(h):
    _check(lib().sf_reset(h), "sf_reset")


def sf_set_stream(h, stream):
    _check(lib().sf_set_stream(h, _stream_handle(stream)), "sf_set_stream")


def sf_insert(h, keys, key_bytes: int = 4):
    p, n = _keys_ptr(keys, key_bytes)
    _check(lib().sf_insert(h, p, n), "sf_insert")


def sf_delete(h, keys, key_bytes: int = 4):
    p, n = _keys_ptr(keys, key_bytes)
    _check(lib().sf_delete(h, p, n), "sf_delete")


def sf_update(h, keys, ops, key_bytes: int = 4):
    import torch
    p, n = _keys_ptr(keys, key_bytes)
    if not (isinstance(ops, torch.Tensor) and ops.is_cuda and ops.dtype == torch.uint8
            and ops.is_contiguous() and ops.numel() == n):
        raise TypeError("ops must be a contiguous GPU uint8 tensor with one entry per key")
    _check(lib().sf_update(h, p, ops.data_ptr(), n), "sf_update")


def sf_query(h, keys, out, key_bytes: int = 4):
    p, n = _keys_ptr(keys, key_bytes)
    if out.numel() < n or out.element_size() != 4 or not out.is_cuda:
        raise ValueError("out must be a GPU 4-byte tensor with one element per key")
    _check(lib().sf_query(h, p, n, out.data_ptr()), "sf_query")


def sf_query_slim(slim, cfg: sf_config, keys, out, stream=None):
    p, n = _keys_ptr(keys, cfg.key_bytes)
    if out.numel() < n or out.element_size() != 4 or not out.is_cuda:
        raise ValueError("out must be a GPU 4-byte tensor with one element per key")
    _check(lib().sf_query_slim(slim.data_ptr(), ctypes.byref(cfg), p, n, out.data_ptr(),
                               _stream_handle(stream)), "sf_query_slim")


def sf_query_slim_noalloc(slim, cfg: sf_config, keys, out, stream=None):
    """sf_query_slim without any allocation: per-row counters in the library's
    static device array (n * d <= NOALLOC_QUERY_COUNTERS)."""
    p, n = _keys_ptr(keys, cfg.key_bytes)
    if out.numel() < n or out.element_size() != 4 or not out.is_cuda:
        raise ValueError("out must be a GPU 4-byte tensor with one element per key")
    _check(lib().sf_query_slim_noalloc(slim.data_ptr(), ctypes.byref(cfg), p, n, out.data_ptr(),
                                       _stream_handle(stream)), "sf_query_slim_noalloc")


def sf_export_slim(h, out):
    _check(lib().sf_export_slim(h, out.ctypes.data if hasattr(out, "ctypes") else out.data_ptr(),
                                out.size if hasattr(out, "ctypes") else out.numel()),
           "sf_export_slim")


def sf_export_fat(h, out):
    _check(lib().sf_export_fat(h, out.ctypes.data if hasattr(out, "ctypes") else out.data_ptr(),
                               out.size if hasattr(out, "ctypes") else out.numel()),
           "sf_export_fat")


def sf_sync(h):
    _check(lib().sf_sync(h), "sf_sync")


def sf_set_tile(h, tile_ops: int):
    _check(lib().sf_set_tile(h, tile_ops), "sf_set_tile")


def sf_profile(h, enable: bool):
    _check(lib().sf_profile(h, int(bool(enable))), "sf_profile")


def sf_profile_read(h, reset: bool = True) -> dict:
    """{kind: (total ms, launches, items)} of the kernels launched while profiling."""
    st = sf_kernel_stats()
    _check(lib().sf_profile_read(h, ctypes.byref(st), int(bool(reset))), "sf_profile_read")
    return {k: (st.ms[i], int(st.launches[i]), int(st.items[i])) for i, k in enumerate(KERNEL_KINDS)}


class Sketch:
    """One SF-sketch on the current GPU.

    d rows; w Slim counters (= Fat buckets) per row; z Fat counters per bucket;
    keys are uint32 (key_bytes=4, torch.int32/uint32 tensors) or packed 13-byte
    strings (key_bytes=13, uint8 tensors); batch_ops is the update schedule's
    batch size (1 = sequential semantics).
    """

    def __init__(self, d: int, w: int, z: int, key_bytes: int = 4, seed_base: int = 1,
                 batch_ops: int = 1 << 20, hbm_budget_bytes: int = 0, stream=None):
        self.cfg = make_config(d, w, z, key_bytes, seed_base, batch_ops)
        self.d, self.w, self.z, self.key_bytes = d, w, z, key_bytes
        self._h = sf_create(self.cfg, hbm_budget_bytes, stream)

    @property
    def footprint(self) -> int:
        return sf_footprint(self.cfg)

    def close(self):
        if getattr(self, "_h", None):
            sf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, keys):
        sf_insert(self._h, keys, self.key_bytes)

    def delete(self, keys):
        sf_delete(self._h, keys, self.key_bytes)

    def update(self, keys, ops):
        sf_update(self._h, keys, ops, self.key_bytes)

    def update_host(self, keys, ops=None, chunk_ops: int = 0):
        """Updates from PINNED host tensors (torch ... pin_memory=True): keys (int32 / uint8
        rows of 13 bytes), ops (uint8, None = all inserts).  chunk_ops: ops per copy chunk,
        a multiple of batch_ops (0: 4 batches).  Returns once the host buffers are free."""
        import torch
        for t, what in ((keys, "keys"), (ops, "ops")):
            if t is not None and (not isinstance(t, torch.Tensor) or t.is_cuda or not t.is_pinned()
                                  or not t.is_contiguous()):
                raise TypeError(f"{what} must be a contiguous pinned host tensor")
        n = keys.numel() * keys.element_size() // self.key_bytes
        if ops is not None and ops.numel() != n:
            raise ValueError("ops must hold one code per key")
        chunk = chunk_ops or 4 * self.cfg.batch_ops
        _check(lib().sf_update_host(self._h, keys.data_ptr(), ops.data_ptr() if ops is not None else None,
                                    n, chunk), "sf_update_host")

    def query(self, keys, out=None):
        import torch
        n = keys.numel() * keys.element_size() // self.key_bytes
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=keys.device)
        sf_query(self._h, keys, out, self.key_bytes)
        return out

    def query_host(self, keys, out=None, streams: int = 4):
        """Queries of keys in pinned host memory through the multi-stream pipeline
        (sf_query_host); answers land in pinned host memory (returned)."""
        import torch
        if not isinstance(keys, torch.Tensor) or keys.is_cuda or not keys.is_pinned():
            raise TypeError("keys must be a pinned host tensor")
        n = keys.numel() * keys.element_size() // self.cfg.key_bytes
        if out is None:
            out = torch.empty(n, dtype=torch.int32).pin_memory()
        if out.numel() < n or out.element_size() != 4:
            raise ValueError("out must hold one 4-byte answer per key")
        _check(lib().sf_query_host(self._h, keys.data_ptr(), n, out.data_ptr(), streams), "sf_query_host")
        return out

    def export_slim(self, out=None):
        import numpy as np
        if out is None:
            out = np.empty((self.d, self.w), dtype=np.uint16)
        sf_export_slim(self._h, out)
        return out

    def export_fat(self, out=None):
        import numpy as np
        if out is None:
            out = np.empty((self.d, self.w, self.z), dtype=np.uint32)
        sf_export_fat(self._h, out)
        return out

    def reset(self):
        sf_reset(self._h)

    def set_tile(self, tile_ops: int):
        sf_set_tile(self._h, tile_ops)

    def merge_stats(self):
        """(insert entries, delete entries) emitted by the batch-wide merge so far."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sf_merge_stats(self._h, ctypes.byref(a), ctypes.byref(b)), "sf_merge_stats")
        return int(a.value), int(b.value)

    def set_merge(self, batch_wide):
        """Merge duplicate keys across the whole batch (True / 1, the default: owner-computes
        S1..S5 for batches of at least w ops where the shape allows), per tile (False / 0),
        across the batch with atomic S1..S5 (2), or with owner-computes for every batch (3)."""
        mode = int(batch_wide) if not isinstance(batch_wide, bool) else int(batch_wide)
        _check(lib().sf_set_merge(self._h, mode), "sf_set_merge")

    def set_owner_range(self, shift: int):
        """Owner path: ranges of 2^shift cells per row (0: the default size)."""
        _check(lib().sf_set_owner_range(self._h, int(shift)), "sf_set_owner_range")

    def owner_range(self) -> int:
        """The owner path's range shift (0 when the shape has no owner path)."""
        rc = lib().sf_owner_range(self._h)
        if rc < 0:
            _check(rc, "sf_owner_range")
        return rc

    def set_streams(self, mode: int):
        """Owner path: partition side of the next batch on a second stream (1), one stream (0),
        or by batch size (-1, the default)."""
        _check(lib().sf_set_streams(self._h, int(mode)), "sf_set_streams")

    def merge_path(self) -> int:
        """0 per-tile merging, 1 batch merge + owner-computes S1..S5 for large batches, 2 batch
        merge + atomic S1..S5, 3 owner-computes for every batch."""
        rc = lib().sf_merge_path(self._h)
        if rc < 0:
            _check(rc, "sf_merge_path")
        return rc

    def profile(self, enable: bool = True):
        sf_profile(self._h, enable)

    def profile_read(self, reset: bool = True) -> dict:
        return sf_profile_read(self._h, reset)

    def sync(self):
        sf_sync(self._h)


# ---------------------------------------------------------------- sketch groups

def _cfg_array(cfgs):
    arr = (sf_config * len(cfgs))()
    for i, c in enumerate(cfgs):
        arr[i] = c if isinstance(c, sf_config) else make_config(**c)
    return arr


def _seg_array(seg, n):
    import numpy as np
    a = np.ascontiguousarray(seg, dtype=np.uint64)
    if a.shape != (n + 1,):
        raise ValueError(f"seg must have n+1 = {n + 1} offsets")
    return a


def sf_group_footprint(cfgs, round_ops: int = 0) -> int:
    arr = _cfg_array(cfgs)
    return int(lib().sf_group_footprint(len(cfgs), arr, round_ops))


class SketchGroup:
    """Many independent sketches updated and queried by the same launches.

    cfgs: one sf_config (or dict of make_config arguments) per sketch.  Keys of a
    call are every sketch's keys concatenated; seg (n+1 host offsets) marks
    where each sketch's keys start.  Each sketch follows its own batch schedule,
    so its state equals a lone Sketch fed the same ops.
    """

    def __init__(self, cfgs, round_ops: int = 0, hbm_budget_bytes: int = 0, stream=None):
        self._arr = _cfg_array(cfgs)
        self.n = len(cfgs)
        self.cfgs = [self._arr[i] for i in range(self.n)]
        self.key_bytes = self.cfgs[0].key_bytes
        h = ctypes.c_void_p()
        _check(lib().sf_group_create(self.n, self._arr, round_ops, hbm_budget_bytes,
                                     _stream_handle(stream), ctypes.byref(h)), "sf_group_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().sf_group_destroy(self._h), "sf_group_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ops_ptr(self, ops, n):
        import torch
        if not (isinstance(ops, torch.Tensor) and ops.is_cuda and ops.dtype == torch.uint8
                and ops.is_contiguous() and ops.numel() == n):
            raise TypeError("ops must be a contiguous GPU uint8 tensor with one entry per key")
        return ops.data_ptr()

    def insert(self, keys, seg):
        p, n = _keys_ptr(keys, self.key_bytes)
        sg = _seg_array(seg, self.n)
        _check(lib().sf_group_insert(self._h, p, sg.ctypes.data), "sf_group_insert")

    def delete(self, keys, seg):
        p, n = _keys_ptr(keys, self.key_bytes)
        sg = _seg_array(seg, self.n)
        _check(lib().sf_group_delete(self._h, p, sg.ctypes.data), "sf_group_delete")

    def update(self, keys, ops, seg):
        p, n = _keys_ptr(keys, self.key_bytes)
        sg = _seg_array(seg, self.n)
        _check(lib().sf_group_update(self._h, p, self._ops_ptr(ops, n), sg.ctypes.data),
               "sf_group_update")

    def query(self, keys, seg, out=None):
        import torch
        p, n = _keys_ptr(keys, self.key_bytes)
        sg = _seg_array(seg, self.n)
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=keys.device)
        if out.numel() < n or out.element_size() != 4 or not out.is_cuda:
            raise ValueError("out must be a GPU 4-byte tensor with one element per key")
        _check(lib().sf_group_query(self._h, p, sg.ctypes.data, out.data_ptr()), "sf_group_query")
        return out

    def export_slim(self, i: int, out=None):
        import numpy as np
        c = self.cfgs[i]
        if out is None:
            out = np.empty((c.d, c.w), dtype=np.uint16)
        ptr, cnt = (out.ctypes.data, out.size) if hasattr(out, "ctypes") else (out.data_ptr(), out.numel())
        _check(lib().sf_group_export_slim(self._h, i, ptr, cnt), "sf_group_export_slim")
        return out

    def export_fat(self, i: int, out=None):
        import numpy as np
        c = self.cfgs[i]
        if out is None:
            out = np.empty((c.d, c.w, c.z), dtype=np.uint32)
        ptr, cnt = (out.ctypes.data, out.size) if hasattr(out, "ctypes") else (out.data_ptr(), out.numel())
        _check(lib().sf_group_export_fat(self._h, i, ptr, cnt), "sf_group_export_fat")
        return out

    def reset(self):
        _check(lib().sf_group_reset(self._h), "sf_group_reset")

    def sync(self):
        _check(lib().sf_group_sync(self._h), "sf_group_sync")

    def set_graph(self, enable: bool):
        _check(lib().sf_group_set_graph(self._h, int(bool(enable))), "sf_group_set_graph")

    def set_tile(self, tile_ops: int):
        _check(lib().sf_group_set_tile(self._h, tile_ops), "sf_group_set_tile")

    def set_merge(self, batch_wide):
        """Merge duplicate (key, sketch) pairs across each sub-round (True / 1, the default:
        owner-computes S1..S5 when every sketch has the same d and z), per tile (False / 0), or
        across each sub-round with atomic S1..S5 (2)."""
        _check(lib().sf_group_set_merge(self._h, int(batch_wide)), "sf_group_set_merge")

    def set_owner_ratio(self, ratio: float):
        """Mode 1: a sketch's batch is owner-computed when it has at least ratio * w ops, else it
        takes the atomic kernels in the same sub-round (0: every batch owner-computed)."""
        _check(lib().sf_group_set_owner_ratio(self._h, float(ratio)), "sf_group_set_owner_ratio")

    def merge_path(self) -> int:
        """0 per-tile merging, 1 batch merge + owner-computes S1..S5, 2 batch merge + atomics."""
        rc = lib().sf_group_merge_path(self._h)
        if rc < 0:
            _check(rc, "sf_group_merge_path")
        return rc

    def merge_stats(self):
        """(insert entries, delete entries) emitted by the batch-wide merge so far, all sketches."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sf_group_merge_stats(self._h, ctypes.byref(a), ctypes.byref(b)), "sf_group_merge_stats")
        return int(a.value), int(b.value)

    def rounds(self):
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sf_group_rounds(self._h, ctypes.byref(a), ctypes.byref(b)), "sf_group_rounds")
        return int(a.value), int(b.value)

    def profile(self, enable: bool = True):
        _check(lib().sf_group_profile(self._h, int(bool(enable))), "sf_group_profile")

    def profile_read(self, reset: bool = True) -> dict:
        st = sf_kernel_stats()
        _check(lib().sf_group_profile_read(self._h, ctypes.byref(st), int(bool(reset))),
               "sf_group_profile_read")
        return {k: (st.ms[i], int(st.launches[i]), int(st.items[i])) for i, k in enumerate(KERNEL_KINDS)}


# ---------------------------------------------------------------- sketch pools (serving)

SF_REQ_INSERT, SF_REQ_DELETE, SF_REQ_UPDATE, SF_REQ_QUERY = 0, 1, 2, 3


class sf_request(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("ops", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("slot", ctypes.c_uint32), ("kind", ctypes.c_uint32)]


def sf_pool_slot_bytes(cfg: sf_config) -> int:
    return int(lib().sf_pool_slot_bytes(ctypes.byref(cfg)))


class SketchPool:
    """Slots of one sketch shape under an HBM budget, launched request by request.

    launch() takes a list of (slot, kind, keys, ops, out) with at most one
    request per slot; it returns a ticket, and done()/wait() report completion.
    """

    def __init__(self, cfg: sf_config, max_slots: int = 0, round_ops: int = 0,
                 hbm_budget_bytes: int = 0, stream=None):
        self.cfg = cfg
        h = ctypes.c_void_p()
        _check(lib().sf_pool_create(ctypes.byref(cfg), max_slots, round_ops, hbm_budget_bytes,
                                    _stream_handle(stream), ctypes.byref(h)), "sf_pool_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().sf_pool_destroy(self._h), "sf_pool_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def capacity(self):
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().sf_pool_capacity(self._h, ctypes.byref(a), ctypes.byref(b)), "sf_pool_capacity")
        return int(a.value), int(b.value)

    def acquire(self):
        """A zeroed slot, or None when the budget holds no free slot."""
        s = ctypes.c_uint32()
        rc = lib().sf_pool_acquire(self._h, ctypes.byref(s))
        if rc == SF_ENOMEM:
            return None
        _check(rc, "sf_pool_acquire")
        return int(s.value)

    def release(self, slot: int):
        _check(lib().sf_pool_release(self._h, slot), "sf_pool_release")

    def launch(self, reqs) -> int:
        """reqs: iterable of (slot, kind, keys_tensor, ops_tensor_or_None, out_tensor_or_None)."""
        reqs = list(reqs)
        arr = (sf_request * max(1, len(reqs)))()
        kb = self.cfg.key_bytes
        for i, (slot, kind, keys, ops, out) in enumerate(reqs):
            p, n = _keys_ptr(keys, kb)
            arr[i] = sf_request(p, ops.data_ptr() if ops is not None else None,
                                out.data_ptr() if out is not None else None, n, slot, kind)
        t = ctypes.c_uint64()
        _check(lib().sf_pool_launch(self._h, arr, len(reqs), ctypes.byref(t)), "sf_pool_launch")
        return int(t.value)

    def done(self, ticket: int) -> bool:
        rc = lib().sf_pool_done(self._h, ticket)
        if rc < 0:
            _check(rc, "sf_pool_done")
        return rc == 1

    def wait(self, ticket: int):
        _check(lib().sf_pool_wait(self._h, ticket), "sf_pool_wait")

    def export_slim(self, slot: int, out=None, asynchronous: bool = False):
        import numpy as np
        c = self.cfg
        if out is None:
            out = np.empty((c.d, c.w), dtype=np.uint16)
        ptr, cnt = (out.ctypes.data, out.size) if hasattr(out, "ctypes") else (out.data_ptr(), out.numel())
        _check(lib().sf_pool_export_slim(self._h, slot, ptr, cnt, int(asynchronous)), "sf_pool_export_slim")
        return out

    def export_fat(self, slot: int, out=None):
        import numpy as np
        c = self.cfg
        if out is None:
            out = np.empty((c.d, c.w, c.z), dtype=np.uint32)
        ptr, cnt = (out.ctypes.data, out.size) if hasattr(out, "ctypes") else (out.data_ptr(), out.numel())
        _check(lib().sf_pool_export_fat(self._h, slot, ptr, cnt), "sf_pool_export_fat")
        return out

    def sync(self):
        _check(lib().sf_pool_sync(self._h), "sf_pool_sync")

    def set_tile(self, tile_ops: int):
        _check(lib().sf_pool_set_tile(self._h, tile_ops), "sf_pool_set_tile")

    def set_merge(self, batch_wide: bool):
        """Merge duplicate (key, slot) pairs across each sub-round (True, the default) or per tile."""
        _check(lib().sf_pool_set_merge(self._h, int(bool(batch_wide))), "sf_pool_set_merge")

    def set_owner_ratio(self, ratio: float):
        """Batches of at least ratio * w ops take the owner-computes path (pools whose slots hold
        at most 64 MiB of records; default 0.5)."""
        _check(lib().sf_pool_set_owner_ratio(self._h, float(ratio)), "sf_pool_set_owner_ratio")

    def merge_stats(self):
        """(insert entries, delete entries) emitted by the batch-wide merge so far, all launches."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sf_pool_merge_stats(self._h, ctypes.byref(a), ctypes.byref(b)), "sf_pool_merge_stats")
        return int(a.value), int(b.value)
