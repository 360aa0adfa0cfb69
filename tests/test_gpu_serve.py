"""Serving loop on the GPU: every stream's result is the same alone and in the
mix (bit-exact), matches the oracle, and admission respects the HBM budget."""
import numpy as np
import pytest

import oracle
import paper_1701_04148_amd as sf
import sfgen
from paper_1701_04148_amd.serve import Server
from tests.gpu_support import assert_same, say

pytestmark = pytest.mark.gpu

CFG = dict(d=4, w=2048, z=4, key_bytes=4, seed_base=1, batch_ops=3000)


def _workload(seed=1, n_streams=40, per_stream=6):
    return sfgen.serving(seed=seed, n_streams=n_streams, per_stream=per_stream, size_range=(50, 9000),
                         pool_keys=1 << 18, universe=20_000, open_window=0.02, stream_rate=400.0)


def _key_fn(w, pool_t):
    """Device keys of a request: a slice of the pool, or (deletes) its pieces joined
    up front, before any pool launch reads them."""
    import torch
    joined = {(r.stream, r.seq): torch.cat([pool_t[o:o + c] for o, c in r.pieces])
              for r in w.requests if r.pieces}
    torch.cuda.synchronize()
    return lambda r: joined[(r.stream, r.seq)] if r.pieces else pool_t[r.off:r.off + r.n]


def _run_mixed(w, max_slots, realtime, max_launch_keys=1 << 15, merge=True, ratio=None):
    import torch
    pool_t = torch.from_numpy(w.pool.view(np.int32)).cuda()
    key_of = _key_fn(w, pool_t)
    outs = {i: torch.full((r.n,), -1, dtype=torch.int32, device="cuda")
            for i, r in enumerate(w.requests) if r.kind == sf.SF_REQ_QUERY}
    index = {id(r): i for i, r in enumerate(w.requests)}
    slims = {s: torch.zeros(CFG["d"] * CFG["w"], dtype=torch.int16, device="cuda")
             for s in range(w.n_streams)}
    pool = sf.SketchPool(sf.make_config(**CFG), max_slots=max_slots)
    pool.set_merge(merge)
    if ratio is not None:
        pool.set_owner_ratio(ratio)
    srv = Server(pool, max_launch_keys=max_launch_keys, max_in_flight=3)
    st = srv.run(w.requests, key_of=key_of,
                 out_of=lambda r: outs[index[id(r)]], export_to=lambda s: slims[s], realtime=realtime)
    pool.sync()
    torch.cuda.synchronize()
    res = {s: slims[s].cpu().numpy().view(np.uint16).reshape(CFG["d"], CFG["w"]) for s in slims}
    ans = {i: o.cpu().numpy().view(np.uint32) for i, o in outs.items()}
    pool.close()
    return st, res, ans


def _run_alone(w, stream):
    import torch
    pool_t = torch.from_numpy(w.pool.view(np.int32)).cuda()
    key_of = _key_fn(w, pool_t)
    pool = sf.SketchPool(sf.make_config(**CFG), max_slots=1)
    slot = pool.acquire()
    ans = {}
    for i, r in enumerate(w.requests):
        if r.stream != stream:
            continue
        out = torch.full((r.n,), -1, dtype=torch.int32, device="cuda") if r.kind == sf.SF_REQ_QUERY else None
        t = pool.launch([(slot, r.kind, key_of(r), None, out)])
        pool.wait(t)
        if out is not None:
            ans[i] = out.cpu().numpy().view(np.uint32)
    slim = pool.export_slim(slot)
    fat = pool.export_fat(slot)
    pool.close()
    return slim, fat, ans


def _oracle_stream(w, stream):
    ref = oracle.Sketch(CFG["d"], CFG["w"], CFG["z"])
    ans = {}
    for i, r in enumerate(w.requests):
        if r.stream != stream:
            continue
        keys = w.keys_of(r)
        if r.kind == sf.SF_REQ_QUERY:
            ans[i] = ref.query(keys)
        else:
            ops = np.full(r.n, 1 if r.kind == sf.SF_REQ_DELETE else 0, np.uint8)
            assert ref.batch(keys, ops, CFG["batch_ops"], checked=True) == 0
    return ref.slim(), ref.fat(), ans


@pytest.mark.parametrize("realtime,merge,ratio", [(False, True, None), (True, True, None), (False, False, None),
                                                  (False, True, 0.0), (False, True, 0.5), (False, True, 1e6)])
def test_alone_equals_mixed_and_oracle(realtime, merge, ratio):
    """A request batch of at least ratio * w ops (default 0.5) takes the owner-computes path, the
    others in its sub-round the atomic kernels; every ratio gives the oracle's state (the lone
    runs keep the default ratio)."""
    w = _workload()
    say(f"[case] serving mix realtime={realtime} merge={merge} ratio={ratio}: {len(w.requests)} requests, "
        f"{w.n_streams} streams")
    st, res, ans = _run_mixed(w, max_slots=8, realtime=realtime, merge=merge, ratio=ratio)
    say(f"  launches {st.launches}, mean {st.mean_requests_per_launch:.1f} req/launch, "
        f"latency {st.latency_ms}, peak resident {st.peak_resident}")
    assert st.peak_resident <= 8 and st.launches > 1 and st.mean_requests_per_launch > 1
    assert all(o.done >= o.issued >= 0 for o in st.outcomes)
    for stream in (0, 1, 7, 23, 39):
        slim_a, fat_a, ans_a = _run_alone(w, stream)
        assert_same(res[stream], slim_a, f"slim of stream {stream}: mixed vs alone")
        for i, a in ans_a.items():
            assert_same(ans[i], a, f"query {i} of stream {stream}: mixed vs alone")
        slim_o, fat_o, ans_o = _oracle_stream(w, stream)
        assert_same(slim_a, slim_o, f"slim of stream {stream} vs oracle")
        assert_same(fat_a, fat_o, f"fat of stream {stream} vs oracle")
        for i, a in ans_o.items():
            assert_same(ans_a[i], a, f"query {i} of stream {stream} vs oracle")


def test_admission_by_budget():
    cfg = sf.make_config(**CFG)
    slot = sf.sf_pool_slot_bytes(cfg)
    probe = sf.SketchPool(cfg, max_slots=1)
    probe.close()
    pool = sf.SketchPool(cfg, hbm_budget_bytes=(1 << 31))  # shared buffers + as many slots as fit
    total, free = pool.capacity()
    assert total >= 1 and free == total
    got = [pool.acquire() for _ in range(total)]
    assert None not in got and pool.acquire() is None       # budget exhausted
    pool.release(got[0])
    assert pool.acquire() == got[0]
    pool.close()
    with pytest.raises(sf.SFError):
        sf.SketchPool(cfg, hbm_budget_bytes=slot)           # no room for the shared buffers
    w = _workload(seed=2, n_streams=20, per_stream=4)
    st, _, _ = _run_mixed(w, max_slots=3, realtime=False)
    assert st.peak_resident <= 3 and st.requests == len(w.requests)


def test_pool_launch_with_more_requests_than_a_subround_holds():
    """1700 small insert requests in one launch: each adds a partial partition
    tile, so the merged sub-round closes on its tile budget; every slot still
    matches the oracle."""
    import torch
    cfg = sf.make_config(4, 64, 4, 4, 1, 1000)
    pool = sf.SketchPool(cfg, max_slots=1700, round_ops=1 << 20)   # sub-rounds of <= 1152 tiles
    rng = np.random.default_rng(5)
    slots = [pool.acquire() for _ in range(1700)]
    keys = [rng.integers(0, 500, int(rng.integers(50, 300))).astype(np.uint32) for _ in slots]
    dk = [torch.from_numpy(k.view(np.int32)).cuda() for k in keys]
    say(f"[case] pool launch of {len(slots)} insert requests")
    t = pool.launch([(sl, sf.SF_REQ_INSERT, k, None, None) for sl, k in zip(slots, dk)])
    pool.wait(t)
    for i in range(0, 1700, 37):
        ref = oracle.Sketch(4, 64, 4)
        assert ref.batch(keys[i], None, 1000, checked=True) == 0
        assert_same(pool.export_fat(slots[i]), ref.fat(), f"fat of slot {i}")
        assert_same(pool.export_slim(slots[i]), ref.slim(), f"slim of slot {i}")
    pool.close()


def test_pool_rejects_bad_requests():
    import torch
    pool = sf.SketchPool(sf.make_config(**CFG), max_slots=2)
    a = pool.acquire()
    keys = torch.arange(100, dtype=torch.int32, device="cuda")
    with pytest.raises(sf.SFError):
        pool.launch([(a, sf.SF_REQ_INSERT, keys, None, None), (a, sf.SF_REQ_INSERT, keys, None, None)])
    with pytest.raises(sf.SFError):
        pool.launch([(1 - a, sf.SF_REQ_INSERT, keys, None, None)])   # slot not acquired
    t = pool.launch([(a, sf.SF_REQ_INSERT, keys, None, None)])
    pool.wait(t)
    assert pool.done(t)
    with pytest.raises(sf.SFError):
        pool.set_owner_ratio(-1.0)
    pool.close()
    big = sf.SketchPool(sf.make_config(8, 1 << 21, 4, 4, 1, 1 << 20), max_slots=1)   # 320 MiB slots
    with pytest.raises(sf.SFError):
        big.set_owner_ratio(1.0)                                                      # no owner path
    big.close()
