"""Checks of the synthetic workload generators (inputs only)."""
import numpy as np

import sfgen
from tests.oracle_support import exact_counts, key_view


def test_deterministic_per_seed():
    a = sfgen.make("t", d=4, w=64, z=4, n_universe=500, n_ops=20000, s=1.0, p_del=0.1, seed=3,
                   n_absent=100)
    b = sfgen.make("t", d=4, w=64, z=4, n_universe=500, n_ops=20000, s=1.0, p_del=0.1, seed=3,
                   n_absent=100)
    c = sfgen.make("t", d=4, w=64, z=4, n_universe=500, n_ops=20000, s=1.0, p_del=0.1, seed=4,
                   n_absent=100)
    assert (a.keys == b.keys).all() and (a.ops == b.ops).all() and (a.queries == b.queries).all()
    assert not (a.keys == c.keys).all()


def test_turnstile_is_strict_and_fraction():
    wl = sfgen.make("t", d=4, w=64, z=4, n_universe=2000, n_ops=100000, s=1.1, p_del=0.1, seed=1)
    sign = np.where(wl.ops == 1, -1, 1)
    kv = key_view(wl.keys)
    u, inv = np.unique(kv, return_inverse=True)
    # running count per key never negative
    order = np.lexsort((np.arange(kv.size), inv))
    run = np.zeros(u.size, np.int64)
    for t in order:          # grouped by key, in stream order within each key
        run[inv[t]] += sign[t]
        assert run[inv[t]] >= 0
    assert abs(wl.ops.mean() - 0.1) < 0.01


def test_universe_distinct_and_absent_absent():
    rng = sfgen.rngs(0)
    uni = sfgen.universe_u32(rng[0], 50000)
    assert np.unique(uni).size == uni.size
    ab = sfgen.absent_u32(rng[3], uni, 20000)
    assert not np.isin(ab, uni).any()
    fl = sfgen.flow_keys(rng[0], 20000)
    assert fl.shape == (20000, 13) and np.unique(key_view(fl)).size == 20000
    af = sfgen.absent_flows(rng[3], fl, 5000)
    assert not np.isin(key_view(af), key_view(fl)).any()


def test_zipf_ranks_shape():
    """Top rank frequency of Zipf(1.0) over 1e5 ranks is 1/H(1e5) ~ 8.3%."""
    r = sfgen.zipf_ranks(np.random.default_rng(0), 100_000, 1.0, 1_000_000)
    assert r.min() >= 0 and r.max() < 100_000
    top = np.mean(r == 0)
    assert abs(top - 1 / np.sum(1.0 / np.arange(1, 100_001))) < 0.002


def test_small_config_shape():
    wl = sfgen.config_small()
    assert wl.keys.dtype == np.uint32 and wl.n_ops == 1_000_000 and wl.ops is None
    assert wl.n_queries == 100_000
    f = exact_counts(wl.keys, None, wl.queries)
    assert f.sum() == 1_000_000


def test_serving_deletes_are_live_occurrences():
    """A delete request removes occurrences that its stream inserted and has not yet
    deleted (strict turnstile), drawn over all of the stream's live insert slices."""
    from collections import Counter
    w = sfgen.serving(seed=3, n_streams=60, per_stream=14, size_range=(20, 400), pool_keys=1 << 14,
                      universe=3000, mix=(0.5, 0.35, 0.15))
    by_stream = {}
    for r in w.requests:
        by_stream.setdefault(r.stream, []).append(r)
    multi_slice = 0
    for reqs in by_stream.values():
        reqs.sort(key=lambda r: r.seq)
        live = Counter()
        slices = []                          # (off, n) of the stream's inserts so far
        for r in reqs:
            keys = w.keys_of(r)
            assert keys.shape[0] == r.n
            if r.kind == 0:
                live.update(keys.tolist())
                slices.append((r.off, r.n))
            elif r.kind == 1:
                assert r.n > 0 and sum(c for _, c in r.pieces) == r.n
                for o, c in r.pieces:        # every piece lies inside one of the stream's inserts
                    assert any(so <= o and o + c <= so + sn for so, sn in slices)
                got = Counter(keys.tolist())
                assert all(live[k] >= v for k, v in got.items())
                live.subtract(got)
                multi_slice += len(r.pieces) > 1
    assert multi_slice > 0                   # deletes reach back past the latest insert
