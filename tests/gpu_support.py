"""Helpers of the GPU parity tests: move seeded inputs to the device, run the
HIP path through the C ABI, run the oracle on the same inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import paper_1701_04148_amd as sf


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_keys(keys: np.ndarray):
    import torch
    if keys.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(keys, dtype=np.uint32).view(np.int32)).cuda()
    return torch.from_numpy(np.ascontiguousarray(keys).reshape(-1)).cuda()


def owner_shape(d, w, z) -> bool:
    """Whether sf_set_merge(1) takes the owner-computes path for this shape (the rule of
    sf.h: ranges of 2^k >= 16 cells, at most min(1024, 8192 / d) per row, at most 8192 Fat
    counters and a 16-bit local code per range)."""
    rmax = min(1024, 16384 // (2 * d))
    zbits = max(0, (z - 1).bit_length())
    sh = 4
    while -(-w // (1 << sh)) > rmax:
        sh += 1
    return (1 << sh) * z <= 8192 and (1 << sh) << zbits <= 65536


def gpu_run(d, w, z, kb, keys, ops, queries, b, seed_base=1, calls=1, merge=1, tile=2048, streams=-1,
            shift=0):
    """Updates (split into `calls` consecutive calls) then queries, on the GPU.
    streams: sf_set_streams mode of the owner path; shift: its range size (sf_set_owner_range,
    0 the default).  Returns (fat, slim, answers)."""
    import torch
    sk = sf.Sketch(d, w, z, key_bytes=kb, seed_base=seed_base, batch_ops=b)
    sk.set_merge(int(merge))
    sk.set_tile(tile)
    sk.set_streams(streams)
    if shift:
        sk.set_owner_range(shift)
        assert sk.owner_range() == shift
    path = sk.merge_path()
    want = int(merge) if int(merge) not in (1, 3) or owner_shape(d, w, z) else 2
    assert path == want, (merge, path, want)
    n = keys.shape[0]
    cuts = np.linspace(0, n, calls + 1).astype(np.int64)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        k = dev_keys(keys[lo:hi])
        if ops is None:
            sk.insert(k)
        else:
            sk.update(k, torch.from_numpy(np.ascontiguousarray(ops[lo:hi])).cuda())
    ans = sk.query(dev_keys(queries)).cpu().numpy().view(np.uint32) if queries.shape[0] else \
        np.zeros(0, np.uint32)
    sk.sync()
    fat, slim = sk.export_fat(), sk.export_slim()
    sk.close()
    return fat, slim, ans


def oracle_run(d, w, z, kb, keys, ops, queries, b, seed_base=1, calls=1):
    ref = oracle.Sketch(d, w, z, kb, seed_base)
    n = keys.shape[0]
    cuts = np.linspace(0, n, calls + 1).astype(np.int64)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        o = None if ops is None else ops[lo:hi]
        assert ref.batch(keys[lo:hi], o, b, checked=True) == 0
    return ref.fat(), ref.slim(), ref.query(queries)


def assert_same(got, exp, what):
    if not np.array_equal(got, exp):
        bad = np.argwhere(got != exp)
        first = tuple(bad[0])
        raise AssertionError(f"{what}: {bad.shape[0]} mismatches, first at {first}: "
                             f"got {got[first]} expected {exp[first]}")
