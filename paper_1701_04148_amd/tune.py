"""Autotuner for the schedule batch size b of one sketch shape, and for the
launch shape of a sketch group.

The batch schedule trades accuracy for throughput: a larger b runs fewer,
larger batches (fewer launches, more duplicate keys merged) but lets more
inserts of a batch read the Slim state from before the batch.  For one
sketch shape (d, w, z) and a sample stream, the tuner runs the GPU path at
every candidate b, measures

* the time of the update and the query of the sample (host clock around
  the sketch's stream, synchronised), and
* the ARE of the answers against the exact counts of the sample
  (|q - f'| / f over queried keys with f > 0, f' = min(f, 65535)),

takes the smallest candidate (w/16) as the stand-in for sequential SF_F
(b = 1 is far too slow to run), and picks the fastest b whose ARE stays within
``rel * ARE_ref + abs_`` (default 1.10x + 1e-3).  Results are cached per
shape and stream class.

A sketch group's merge path and launch-round size (how many ops one
partition / merge / S1..S5 pass covers) change its speed, never its state:
tune_group times whole update calls of the group's streams for every
candidate and keeps the fastest.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import Sketch, SketchGroup

SLIM_MAX = 65535
BATCH_CAP = 1 << 23


def batch_for_width(w: int) -> int:
    """Default schedule batch size for a sketch of Slim width w: b = min(16 w, 2^23).
    It comes from the oracle's ARE of the batch schedule against sequential SF_F on
    the benchmark workloads under the tolerance ARE <= 1.10 x ARE_seq + 1e-3
    (``python -m oracle.accuracy`` prints the table): on the 1M-insert workload
    (w = 2^14) b = 16 w is within it and 64 w is not; on the 32M-op workload
    (w = 2^20) 2^23 is within it at every skew, 2^24 at Zipf 0.6 only through the
    absolute term, hence the cap."""
    return int(min(16 * w, BATCH_CAP))


def exact_counts(keys: np.ndarray, ops: np.ndarray | None, queries: np.ndarray) -> np.ndarray:
    """Net count of every query key in the stream (inserts minus deletes), on the host.
    keys / queries: uint32 [n] or uint8 [n, 13]."""
    def as_rows(a):
        return a if a.ndim == 1 else np.ascontiguousarray(a).view(np.dtype((np.void, a.shape[1]))).ravel()
    k, q = as_rows(keys), as_rows(queries)
    uniq, inv = np.unique(k, return_inverse=True)
    sign = np.ones(k.shape[0], np.int64) if ops is None else np.where(ops == 1, -1, 1)
    cnt = np.bincount(inv.ravel(), weights=sign, minlength=uniq.shape[0]).astype(np.int64)
    pos = np.searchsorted(uniq, q)
    pos[pos >= uniq.shape[0]] = 0
    return np.where(uniq[pos] == q, cnt[pos], 0)


def are(answers: np.ndarray, f: np.ndarray) -> float:
    """Average relative error over keys with f > 0 (Slim saturation taken into account)."""
    m = f > 0
    if not m.any():
        return 0.0
    a = answers.astype(np.int64)[m]
    fp = np.minimum(f[m], SLIM_MAX)
    return float(np.mean(np.abs(a - fp) / f[m]))


@dataclass
class TuneResult:
    b: int
    ref_b: int
    ref_are: float
    bound: float
    table: list = field(default_factory=list)   # (b, are, ms, feasible, merge mode, range shift) per candidate
    mode: int = 1                                # merge mode (sf_set_merge) of the pick
    shift: int = 0                               # owner range shift (sf_set_owner_range) of the pick, 0: none


def candidates_for(w: int, n_ops: int, cap: int = 1 << 23) -> list[int]:
    """Every power of two from w/16 up to min(64 w, cap), stopping at the first
    one that holds the whole sample (larger ones behave the same on it)."""
    lo = max(64, w // 16)
    out, b = [], 1 << (lo - 1).bit_length()
    while b <= min(64 * w, cap):
        out.append(b)
        if b >= n_ops:
            break
        b <<= 1
    return out or [min(lo, cap)]


def tune_batch(d: int, w: int, z: int, keys: np.ndarray, ops: np.ndarray | None, queries: np.ndarray,
               key_bytes: int = 4, candidates=None, rel: float = 1.10, abs_: float = 1e-3,
               reps: int = 2, modes=(1,), ref_are: float | None = None, shifts=(0,)) -> TuneResult:
    """Pick b (and, among `modes`, the sf_set_merge path, and among `shifts`, the owner
    path's range size: 0 the default, or every allowed one with None) for sketches of
    shape (d, w, z) fed streams like (keys, ops).  Every mode and range size gives the
    same answers, so the accuracy depends on b alone; each candidate keeps its fastest
    launch shape.  ref_are: the sequential ARE of the sample when the caller has it (the
    bound is then taken from it instead of the smallest candidate's)."""
    import torch
    cands = sorted(candidates or candidates_for(w, keys.shape[0]))
    f = exact_counts(keys, ops, queries)
    dev = torch.device("cuda")
    if key_bytes == 4:
        dk = torch.from_numpy(np.ascontiguousarray(keys, np.uint32).view(np.int32)).to(dev)
        dq = torch.from_numpy(np.ascontiguousarray(queries, np.uint32).view(np.int32)).to(dev)
    else:
        dk = torch.from_numpy(np.ascontiguousarray(keys).reshape(-1)).to(dev)
        dq = torch.from_numpy(np.ascontiguousarray(queries).reshape(-1)).to(dev)
    dops = None if ops is None else torch.from_numpy(np.ascontiguousarray(ops)).to(dev)
    out = torch.empty(queries.shape[0], dtype=torch.int32, device=dev)
    rows = []
    for b in cands:
        sk = Sketch(d, w, z, key_bytes=key_bytes, batch_ops=b)
        best, best_mode, best_shift, ans = float("inf"), modes[0], 0, None
        for mode in modes:
            sk.set_merge(mode)
            owner = sk.merge_path() in (1, 3)
            for shift in (owner_shifts(sk) if shifts is None else shifts) if owner else (0,):
                if owner:
                    sk.set_owner_range(shift)
                for _ in range(reps):
                    sk.reset()
                    sk.sync()
                    t0 = time.perf_counter()
                    if dops is None:
                        sk.insert(dk)
                    else:
                        sk.update(dk, dops)
                    sk.query(dq, out)
                    sk.sync()
                    ms = (time.perf_counter() - t0) * 1e3
                    if ms < best:
                        best, best_mode, best_shift = ms, sk.merge_path(), sk.owner_range() if owner else 0
                if ans is None:
                    ans = out.cpu().numpy().view(np.uint32)
            if owner:
                sk.set_owner_range(0)
        rows.append([b, are(ans, f), best, None, best_mode, best_shift])
        sk.close()
    ref_b = rows[0][0]
    if ref_are is None:
        ref_are = rows[0][1]
    bound = rel * ref_are + abs_
    for r in rows:
        r[3] = r[1] <= bound
    feasible = [r for r in rows if r[3]]
    best_row = min(feasible, key=lambda r: r[2]) if feasible else rows[0]
    return TuneResult(best_row[0], ref_b, ref_are, bound, rows, best_row[4], best_row[5])


def owner_shifts(sk) -> list[int]:
    """Every range shift sf_set_owner_range accepts for this sketch's shape."""
    from . import SFError
    out = []
    for shift in range(4, 24):
        try:
            sk.set_owner_range(shift)
        except SFError:
            continue
        out.append(shift)
    sk.set_owner_range(0)
    return out


class Autotuner:
    """Per-shape cache of tune_batch results (key: d, w, z, key_bytes, stream class)."""

    def __init__(self, **kw):
        self.kw = kw
        self.cache: dict = {}

    def batch_for(self, d, w, z, keys, ops, queries, key_bytes=4, stream_class="default") -> TuneResult:
        k = (d, w, z, key_bytes, stream_class)
        if k not in self.cache:
            self.cache[k] = tune_batch(d, w, z, keys, ops, queries, key_bytes=key_bytes, **self.kw)
        return self.cache[k]


@dataclass
class GroupShape:
    mode: int                                   # sf_group_set_merge mode of the pick
    round_ops: int                              # ops per launch round of the pick
    ms: float                                   # its fastest update call
    table: list = field(default_factory=list)   # (mode, ratio, round_ops, ms, sub-rounds) per candidate
    ratio: float = 0.0                          # sf_group_set_owner_ratio of the pick (mode 1)


def group_round_candidates(cfgs, caps=(1 << 22, 1 << 23, 1 << 24)) -> list[int]:
    """Round sizes to try: each cap that holds the largest batch of any sketch (a batch is
    never split over rounds), at least one."""
    max_b = max(int(c.batch_ops) for c in cfgs)
    out = sorted({max(c, max_b) for c in caps})
    return out


def tune_group(cfgs, keys, ops, seg, modes=(1, 2), ratios=(0.0, 0.5, 1.0, 2.0), round_ops=None,
               reps=2) -> GroupShape:
    """Pick the merge path (among `modes`; for mode 1 also the owner ratio among `ratios`)
    and the launch-round size of a group of sketches `cfgs` fed the device streams (keys,
    ops) cut by the host offsets seg, by timing one update call per repetition (after one
    untimed call that also records the graph)."""
    import torch
    rows = []
    for r in round_ops or group_round_candidates(cfgs):
        G = SketchGroup(cfgs, round_ops=r)
        for mode in modes:
            G.set_merge(mode)
            for ratio in (ratios if G.merge_path() == 1 else (0.0,)):
                if G.merge_path() == 1:
                    G.set_owner_ratio(ratio)
                best = float("inf")
                for i in range(reps + 1):
                    G.reset()
                    G.sync()
                    t0 = time.perf_counter()
                    G.update(keys, ops, seg)
                    G.sync()
                    if i:
                        best = min(best, (time.perf_counter() - t0) * 1e3)
                rows.append([G.merge_path(), float(ratio), int(r), best, G.rounds()[0]])
        G.close()
        del G
        torch.cuda.empty_cache()
    pick = min(rows, key=lambda x: x[3])
    return GroupShape(pick[0], pick[2], pick[3], rows, pick[1])
