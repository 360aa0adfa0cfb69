"""Seeded synthetic workloads for the SF-sketch hot path.

This module only draws inputs: key universes, Zipf-ranked streams with
turnstile deletions, absent query keys.  It holds none of the sketch's
arithmetic, so both the CPU oracle and the HIP path consume its output.

The paper evaluates on YCSB uniform / zipf-0.99 item streams and on a campus
gateway trace (Section 5); none of those are available, so these seeded
generators stand in for them with the same shapes: a universe of distinct
keys, Zipf(s) occurrence counts, a fraction of deletions of previously
inserted occurrences, and queries over present and absent keys.

Recipe (all draws from ``numpy.random.default_rng`` children of
``SeedSequence(seed)``: child 0 universe, 1 ranks, 2 delete flags and
victims, 3 absent keys):

* Zipf(s) over n ranks: P(r) proportional to r^-s, r = 1..n, sampled by
  inverse CDF (float64 cumulative weights, searchsorted of uniform doubles).
* Universe: n distinct keys drawn uniformly (uint32, or 13 random bytes for
  flow keys), shuffled; rank r maps to universe[r].
* Deletions: each op position is a delete candidate with probability p_del;
  a candidate deletes a uniformly chosen live occurrence (swap-remove pool),
  or inserts when nothing is live.  The stream is therefore strict-turnstile.
* Absent keys: uniform keys not in the universe.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsfgen.so")
_lib = None


def build() -> str:
    """Compile the sequential turnstile helper (plain C, gcc)."""
    src = os.path.join(_HERE, "turnstile.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src])
    os.replace(tmp, _SO)
    return _SO


def _native():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.sfgen_turnstile.restype = ctypes.c_int64
        lib.sfgen_turnstile.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def rngs(seed: int, k: int = 4):
    """Independent generators: 0 universe, 1 ranks, 2 deletions, 3 absent keys."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def zipf_ranks(rng: np.random.Generator, n: int, s: float, size: int,
               threaded: bool = True) -> np.ndarray:
    """0-based ranks with P(r) proportional to (r+1)^-s, by inverse CDF.
    threaded: use torch's multi-threaded CPU searchsorted (same indices)."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(size)
    r = None
    if threaded:
        try:
            import torch
            r = torch.searchsorted(torch.from_numpy(cdf), torch.from_numpy(u), right=True).numpy()
        except Exception:  # pragma: no cover
            r = None
    if r is None:
        r = np.searchsorted(cdf, u, side="right")
    return np.minimum(r, n - 1).astype(np.int64)


def universe_u32(rng: np.random.Generator, n: int) -> np.ndarray:
    """n distinct uint32 keys, uniform without replacement, shuffled."""
    keys = np.unique(rng.integers(0, 2**32, size=int(n * 1.05) + 16, dtype=np.uint64))
    while keys.size < n:
        more = rng.integers(0, 2**32, size=n - keys.size + 16, dtype=np.uint64)
        keys = np.unique(np.concatenate([keys, more]))
    keys = keys[:n].astype(np.uint32)
    rng.shuffle(keys)
    return keys


def absent_u32(rng: np.random.Generator, universe: np.ndarray, m: int) -> np.ndarray:
    """m uniform uint32 keys that are not in the universe (may repeat)."""
    out = np.empty(0, dtype=np.uint32)
    while out.size < m:
        cand = rng.integers(0, 2**32, size=m - out.size + 64, dtype=np.uint64).astype(np.uint32)
        cand = cand[~np.isin(cand, universe)]
        out = np.concatenate([out, cand])
    return out[:m]


def _rows_unique(a: np.ndarray) -> bool:
    v = np.ascontiguousarray(a).view(np.dtype((np.void, a.shape[1]))).ravel()
    return np.unique(v).size == v.size


def flow_keys(rng: np.random.Generator, n: int) -> np.ndarray:
    """n distinct 13-byte keys of uniform random bytes, shape (n, 13) uint8."""
    keys = rng.integers(0, 256, size=(n, 13), dtype=np.uint8)
    while not _rows_unique(keys):  # probability ~ n^2 / 2^105: never in practice
        keys = rng.integers(0, 256, size=(n, 13), dtype=np.uint8)
    return keys


def absent_flows(rng: np.random.Generator, universe: np.ndarray, m: int) -> np.ndarray:
    """m uniform 13-byte keys not in the universe."""
    out = rng.integers(0, 256, size=(m, 13), dtype=np.uint8)
    uv = np.ascontiguousarray(universe).view(np.dtype((np.void, 13))).ravel()
    ov = out.view(np.dtype((np.void, 13))).ravel()
    bad = np.isin(ov, uv)
    while bad.any():
        out[bad] = rng.integers(0, 256, size=(int(bad.sum()), 13), dtype=np.uint8)
        ov = out.view(np.dtype((np.void, 13))).ravel()
        bad = np.isin(ov, uv)
    return out


def turnstile(ins_keys: np.ndarray, rng: np.random.Generator, p_del: float):
    """Turn pre-drawn insert keys into a strict-turnstile op stream.

    Returns (keys, ops) with ops 0 = insert, 1 = delete.
    """
    n = ins_keys.shape[0]
    kb = 4 if ins_keys.ndim == 1 else ins_keys.shape[1]
    if p_del <= 0.0:
        return ins_keys.copy(), np.zeros(n, dtype=np.uint8)
    cand = (rng.random(n) < p_del).astype(np.uint8)
    u = rng.random(int(cand.sum()))
    src = np.ascontiguousarray(ins_keys)
    keys = np.empty_like(src)
    ops = np.empty(n, dtype=np.uint8)
    pool = np.empty_like(src)
    _native().sfgen_turnstile(src.ctypes.data, n, kb, cand.ctypes.data, u.ctypes.data,
                              keys.ctypes.data, ops.ctypes.data, pool.ctypes.data)
    return keys, ops


@dataclass
class Workload:
    """One sketch's synthetic input: its shape, op stream and query keys."""
    name: str
    d: int
    w: int
    z: int
    key_bytes: int
    seed_base: int
    keys: np.ndarray             # uint32 [n] or uint8 [n, 13]
    ops: np.ndarray | None       # uint8 [n] (0 insert, 1 delete) or None = all inserts
    queries: np.ndarray          # same key format
    universe: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_ops(self) -> int:
        return int(self.keys.shape[0])

    @property
    def n_queries(self) -> int:
        return int(self.queries.shape[0])


def make(name: str, *, d: int, w: int, z: int, n_universe: int, n_ops: int, s: float,
         p_del: float = 0.0, key_bytes: int = 4, seed: int = 0, seed_base: int = 1,
         n_absent: int = 0, query_universe: bool = True) -> Workload:
    """Generic recipe: universe, Zipf(s) stream of n_ops, optional deletions, queries."""
    g_uni, g_rank, g_del, g_abs = rngs(seed)
    if key_bytes == 4:
        uni = universe_u32(g_uni, n_universe)
    elif key_bytes == 13:
        uni = flow_keys(g_uni, n_universe)
    else:
        raise ValueError("key_bytes must be 4 or 13")
    ranks = zipf_ranks(g_rank, n_universe, s, n_ops)
    ins = uni[ranks]
    keys, ops = turnstile(ins, g_del, p_del)
    # exact occurrence count of every universe key (insert-only streams)
    counts = np.bincount(ranks, minlength=n_universe) if p_del <= 0 else None
    parts = [uni] if query_universe else []
    if n_absent:
        parts.append(absent_u32(g_abs, uni, n_absent) if key_bytes == 4
                     else absent_flows(g_abs, uni, n_absent))
    queries = np.concatenate(parts) if parts else uni[:0]
    return Workload(name, d, w, z, key_bytes, seed_base, np.ascontiguousarray(keys),
                    ops if p_del > 0 else None, np.ascontiguousarray(queries), uni,
                    dict(n_universe=n_universe, n_ops=n_ops, s=s, p_del=p_del, seed=seed,
                         n_absent=n_absent, universe_counts=counts))


# ---- the benchmark configurations -----------------------------------------

def config_small(seed: int = 0) -> Workload:
    """One sketch, d=4, Fat 4x65536 u32, Slim 4x16384 u16; 1M Zipf(1.0) inserts over
    100K distinct uint32 keys; query all 100K."""
    return make("c1_d4_w16384_z4_1M_zipf1.0", d=4, w=16384, z=4, n_universe=100_000,
                n_ops=1_000_000, s=1.0, seed=seed)


def config_main(s: float = 1.0, seed: int = 0, scale: int = 1) -> Workload:
    """One sketch, d=4, Fat 4x2^22 u32, Slim 4x2^20 u16; 32M ops Zipf(s) over 1M distinct
    keys with 10% deletions of live occurrences; query all 1M plus 1M absent keys.
    ``scale`` divides every size (keeps z=4) for quick runs."""
    return make(f"c2_d4_w{2**20 // scale}_z4_{32 // scale}M_zipf{s}_del10",
                d=4, w=2**20 // scale, z=4, n_universe=1_000_000 // scale,
                n_ops=32_000_000 // scale, s=s, p_del=0.10, seed=seed,
                n_absent=1_000_000 // scale)


def config_flows(seed: int = 0, scale: int = 1) -> Workload:
    """One sketch, d=8 over 13-byte flow keys; Fat 8x2^23 u32, Slim 8x2^21 u16;
    128M packets, Zipf(1.2) flow sizes over 4M flows, insert-only; query 4M flows +
    12M absent keys (16M)."""
    return make(f"c3_d8_w{2**21 // scale}_z4_{128 // scale}M_flows_zipf1.2",
                d=8, w=2**21 // scale, z=4, n_universe=4_000_000 // scale,
                n_ops=128_000_000 // scale, s=1.2, key_bytes=13, seed=seed,
                n_absent=12_000_000 // scale)


@dataclass
class MultiWorkload:
    """Many sketches' inputs, concatenated sketch by sketch.

    keys / ops / queries hold every sketch's arrays back to back; seg and qseg
    (n+1 offsets) mark where sketch i's ops and queries start.  w[i] is sketch
    i's Slim width (Fat width = 4 w[i])."""
    name: str
    d: int
    z: int
    w: np.ndarray
    keys: np.ndarray
    ops: np.ndarray
    seg: np.ndarray
    queries: np.ndarray
    qseg: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.w.shape[0])

    def part(self, i: int):
        lo, hi = int(self.seg[i]), int(self.seg[i + 1])
        qlo, qhi = int(self.qseg[i]), int(self.qseg[i + 1])
        return self.keys[lo:hi], self.ops[lo:hi], self.queries[qlo:qhi]


def _multi_sketch(args):
    """One sketch's (keys, ops, queries) of the many-sketch recipe."""
    child, L, s, p_del = args
    g_uni, g_rank, g_del, _ = [np.random.default_rng(c) for c in child.spawn(4)]
    n_uni = max(1, -(-L // 10))
    uni = universe_u32(g_uni, n_uni)
    k, o = turnstile(uni[zipf_ranks(g_rank, n_uni, s, L, threaded=False)], g_del, p_del)
    return k, o, uni


def config_multi(seed: int = 0, n_sketches: int = 1024, length_scale: float = 1.0,
                 d: int = 4, fat_log2=(14, 20), median: float = 200_000.0, sigma: float = 1.0,
                 len_range=(10_000, 4_000_000), s: float = 1.1, p_del: float = 0.05,
                 workers: int = 1) -> MultiWorkload:
    """1024 independent sketches (one per monitoring node): Fat width 2^14..2^20
    uint32 log-uniform per sketch (Slim width a quarter of it, z = 4); stream
    length lognormal (median 200K, sigma 1.0) clipped to [10K, 4M]; universe of
    ceil(length / 10) distinct uint32 keys per stream; Zipf(1.1); 5% deletions
    of live occurrences; queries = each stream's universe.  length_scale
    shrinks every stream (tests).  workers > 1 draws sketches in that many
    freshly started worker processes (same result)."""
    top = np.random.SeedSequence(seed)
    g_shape = np.random.default_rng(top.spawn(1)[0])
    e_fat = g_shape.integers(fat_log2[0], fat_log2[1] + 1, size=n_sketches)
    lens = np.exp(np.log(median) + sigma * g_shape.standard_normal(n_sketches))
    lens = np.clip(np.round(lens), len_range[0], len_range[1])
    lens = np.maximum(1, np.round(lens * length_scale)).astype(np.int64)
    w = (2 ** (e_fat - 2)).astype(np.int64)
    children = np.random.SeedSequence(seed + 1).spawn(n_sketches)
    jobs = [(children[i], int(lens[i]), s, p_del) for i in range(n_sketches)]
    if workers > 1:
        import multiprocessing as mp
        _native()  # build / load the helper once, before forking
        with mp.get_context("spawn").Pool(workers) as pool:
            parts = pool.map(_multi_sketch, jobs, chunksize=max(1, n_sketches // (4 * workers)))
    else:
        parts = [_multi_sketch(j) for j in jobs]
    seg = np.zeros(n_sketches + 1, dtype=np.uint64)
    qseg = np.zeros(n_sketches + 1, dtype=np.uint64)
    seg[1:] = np.cumsum([p[0].shape[0] for p in parts])
    qseg[1:] = np.cumsum([p[2].shape[0] for p in parts])
    return MultiWorkload(f"multi{n_sketches}_d{d}_fat2^{fat_log2[0]}-2^{fat_log2[1]}_lognormal",
                         d, 4, w, np.concatenate([p[0] for p in parts]),
                         np.concatenate([p[1] for p in parts]), seg,
                         np.concatenate([p[2] for p in parts]), qseg,
                         dict(seed=seed, s=s, p_del=p_del, median=median, sigma=sigma,
                              length_scale=length_scale))


@dataclass
class ServeRequest:
    """One request of the serving workload: keys are pool[off : off + n], or for a
    delete the concatenation of pool[o : o + c] over its pieces (o, c)."""
    stream: int
    seq: int          # position in the stream's request order
    kind: int         # 0 insert, 1 delete, 3 query (the sf_request kinds)
    off: int
    n: int
    arrival: float    # seconds after the start
    last: bool        # the stream closes after this request
    pieces: tuple = None  # delete: ((off, count), ...) slices of the pool, in order


@dataclass
class ServeWorkload:
    pool: np.ndarray                # uint32 key pool every request slices
    requests: list                  # ServeRequest, sorted by arrival
    n_streams: int
    meta: dict = field(default_factory=dict)

    def keys_of(self, r: ServeRequest) -> np.ndarray:
        """The request's keys, in order."""
        if r.pieces:
            return np.concatenate([self.pool[o:o + c] for o, c in r.pieces])
        return self.pool[r.off:r.off + r.n]


def serving(seed: int = 0, n_streams: int = 4096, per_stream: int = 16, mix=(0.7, 0.1, 0.2),
            size_range=(1_000, 1_000_000), pool_keys: int = 1 << 26, universe: int = 1_000_000,
            s: float = 1.0, open_window: float = 1.0, stream_rate: float = 16.0) -> ServeWorkload:
    """Request stream of the serving loop.

    Every stream opens at a uniform time in [0, open_window) seconds and then
    issues per_stream requests with exponential gaps (Poisson, stream_rate
    requests/s); its last request closes it.  Kinds insert / delete / query
    with probabilities mix (a delete with nothing live becomes an insert);
    sizes log-uniform in size_range.  Keys come from one pool of pool_keys
    Zipf(s) draws over a universe of distinct uint32: an insert or query takes
    a random slice of the pool.  A delete removes n occurrences drawn uniformly
    from the stream's live ones (all occurrences inserted and not yet deleted;
    n is capped at their number, so the stream stays strict-turnstile): the
    number taken from each live insert slice is multivariate hypergeometric,
    and inside a slice they are its last live positions -- the pool's draws
    are independent and identically distributed, so which positions of a
    slice go does not change the distribution of the deleted keys.  Scale
    offered load with open_window and stream_rate."""
    g_uni, g_rank, g_req, g_arr = rngs(seed)
    uni = universe_u32(g_uni, universe)
    pool = uni[zipf_ranks(g_rank, universe, s, pool_keys)]
    lo, hi = np.log(size_range[0]), np.log(size_range[1])
    reqs = []
    for st in range(n_streams):
        t = float(g_arr.random() * open_window)
        live = []  # [off, remaining] of this stream's inserts
        for q in range(per_stream):
            t += float(g_arr.exponential(1.0 / stream_rate))
            n = int(round(np.exp(lo + (hi - lo) * g_req.random())))
            u = g_req.random()
            kind = 0 if u < mix[0] else (1 if u < mix[0] + mix[1] else 3)
            live = [iv for iv in live if iv[1] > 0]
            if kind == 1 and not live:
                kind = 0
            pieces = None
            if kind == 1:
                rem = np.array([iv[1] for iv in live], dtype=np.int64)
                n = int(min(n, rem.sum()))
                take = g_req.multivariate_hypergeometric(rem, n)
                pieces = []
                for iv, c in zip(live, take):
                    if c:
                        iv[1] -= int(c)
                        pieces.append((iv[0] + iv[1], int(c)))   # the slice's last live positions
                pieces = tuple(pieces)
                off = pieces[0][0]
            else:
                off = int(g_req.integers(0, pool_keys - n + 1))
                if kind == 0:
                    live.append([off, n])
            reqs.append(ServeRequest(st, q, kind, off, n, t, q == per_stream - 1, pieces))
    reqs.sort(key=lambda r: (r.arrival, r.stream, r.seq))
    return ServeWorkload(pool, reqs, n_streams,
                         dict(seed=seed, per_stream=per_stream, mix=mix, size_range=size_range,
                              pool_keys=pool_keys, universe=universe, s=s, open_window=open_window,
                              stream_rate=stream_rate))
