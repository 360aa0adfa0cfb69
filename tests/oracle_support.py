"""Helpers shared by the CPU pin tests: independent hashing and exact counts.

Indices here come from scikit-learn's MurmurHash3_x86_32, not from the C
oracle, so a wrong hash or index split in the oracle shows up as a mismatch.
"""
from __future__ import annotations

import numpy as np
from sklearn.utils import murmurhash3_32


def sk_hash(keys: np.ndarray, seed: int) -> np.ndarray:
    """Row hash of every key as uint32 (uint32 keys: 4 little-endian bytes)."""
    if keys.ndim == 1:
        v = np.ascontiguousarray(keys.astype("<u4")).view("<i4")
        return np.asarray(murmurhash3_32(v, seed=seed, positive=True), dtype=np.uint64).astype(np.uint32)
    return np.array([murmurhash3_32(bytes(k), seed=seed, positive=True) for k in keys], dtype=np.uint32)


def sk_indices(keys: np.ndarray, d: int, w: int, z: int, seed_base: int = 1):
    """(h, f) per key and row, [n][d], by Eq. (1) read 0-based."""
    n = keys.shape[0]
    h = np.empty((n, d), dtype=np.uint32)
    f = np.empty((n, d), dtype=np.uint32)
    for i in range(d):
        c = sk_hash(keys, seed_base + i).astype(np.uint64) % np.uint64(w * z)
        h[:, i] = (c % np.uint64(w)).astype(np.uint32)
        f[:, i] = (c // np.uint64(w)).astype(np.uint32)
    return h, f


def histogram_fat(h, f, ops, d, w, z) -> np.ndarray:
    """Fat as a plain signed histogram of the stream (wraps like uint32)."""
    sign = np.ones(h.shape[0], dtype=np.int64) if ops is None else np.where(ops == 1, -1, 1)
    out = np.zeros((d, w, z), dtype=np.int64)
    for i in range(d):
        np.add.at(out[i], (h[:, i].astype(np.int64), f[:, i].astype(np.int64)), sign)
    return (out % (1 << 32)).astype(np.uint32)


def key_view(keys: np.ndarray) -> np.ndarray:
    if keys.ndim == 1:
        return keys
    return np.ascontiguousarray(keys).view(np.dtype((np.void, keys.shape[1]))).ravel()


def exact_counts(keys, ops, queries) -> np.ndarray:
    """Net frequency f(e) of every query key (0 when absent)."""
    kv, qv = key_view(keys), key_view(queries)
    u, inv = np.unique(kv, return_inverse=True)
    sign = np.ones(kv.shape[0], dtype=np.int64) if ops is None else np.where(ops == 1, -1, 1)
    cnt = np.zeros(u.shape[0], dtype=np.int64)
    np.add.at(cnt, inv.ravel(), sign)
    pos = np.searchsorted(u, qv)
    pos_c = np.minimum(pos, max(u.shape[0] - 1, 0))
    hit = (pos < u.shape[0]) & (u[pos_c] == qv) if u.shape[0] else np.zeros(qv.shape[0], bool)
    return np.where(hit, cnt[pos_c], 0)


def random_turnstile(rng, n_ops, n_keys, p_del, key_bytes=4):
    """Tiny strict-turnstile stream over a small key universe (pure numpy/python)."""
    if key_bytes == 4:
        uni = rng.choice(2**32, size=n_keys, replace=False).astype(np.uint32)
    else:
        uni = rng.integers(0, 256, size=(n_keys, key_bytes), dtype=np.uint8)
    keys = []
    ops = np.zeros(n_ops, dtype=np.uint8)
    live = []
    for t in range(n_ops):
        if live and rng.random() < p_del:
            j = int(rng.integers(len(live)))
            keys.append(live[j])
            live[j] = live[-1]
            live.pop()
            ops[t] = 1
        else:
            k = int(rng.integers(n_keys))
            keys.append(k)
            live.append(k)
    return uni[np.array(keys, dtype=np.int64)], ops, uni
