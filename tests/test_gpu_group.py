"""Sketch groups on the GPU: every sketch of a group must end in exactly the
state the oracle (and a lone sketch) reaches on its own ops with its own
batch size, whatever the round packing, graph capture or tile size."""
import numpy as np
import pytest

import oracle
import paper_1701_04148_amd as sf
import sfgen
from tests.gpu_support import assert_same, dev_keys, say

pytestmark = pytest.mark.gpu


def _cfgs(w, d, batch, kb=4, seeds=None):
    return [sf.make_config(int(d[i]), int(w[i]), 4, kb, int(seeds[i]) if seeds is not None else 1,
                           int(batch[i])) for i in range(len(w))]


def _oracle_parts(m, cfgs, kb=4):
    out = []
    for i, c in enumerate(cfgs):
        k, o, q = m.part(i)
        ref = oracle.Sketch(c.d, c.w, c.z, kb, c.seed_base)
        assert ref.batch(k, o, c.batch_ops, checked=True) == 0
        out.append((ref.fat(), ref.slim(), ref.query(q)))
    return out


def _check_group(G, m, refs):
    import torch
    out = G.query(dev_keys(m.queries), m.qseg)
    G.sync()
    ans = out.cpu().numpy().view(np.uint32)
    for i in range(m.n):
        assert_same(G.export_fat(i), refs[i][0], f"fat of sketch {i}")
        assert_same(G.export_slim(i), refs[i][1], f"slim of sketch {i}")
        assert_same(ans[int(m.qseg[i]):int(m.qseg[i + 1])], refs[i][2], f"queries of sketch {i}")


@pytest.mark.parametrize("merge,ratio", [(1, 0.0), (1, 1.0), (1, 8.0), (1, 1e6), (2, 0.0), (0, 0.0)])
@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("round_ops", [0, 20_000])
def test_group_matches_oracle_per_sketch(graph, round_ops, merge, ratio):
    """48 sketches of different widths, stream lengths and batch sizes, mixed ops; owner-
    computes (1) -- every batch (ratio 0), batches of at least ratio * w ops with the others on
    the atomic kernels in the same sub-rounds, or none (ratio 1e6) --, atomic (2) and per-tile (0)
    merge paths."""
    import torch
    m = sfgen.config_multi(seed=3, n_sketches=48, length_scale=0.03, fat_log2=(8, 13))
    rng = np.random.default_rng(1)
    batch = rng.choice([700, 2048, 5000, 1 << 20], size=m.n)
    cfgs = _cfgs(m.w, np.full(m.n, 4), batch)
    say(f"[case] group n={m.n} ops={m.keys.size} graph={graph} round_ops={round_ops} merge={merge} "
        f"ratio={ratio}")
    G = sf.SketchGroup(cfgs, round_ops=round_ops)
    G.set_graph(graph)
    G.set_merge(merge)
    assert G.merge_path() == merge
    if merge == 1:
        G.set_owner_ratio(ratio)
    G.update(dev_keys(m.keys), torch.from_numpy(m.ops).cuda(), m.seg)
    sub, tiles = G.rounds()
    say(f"  sub-rounds {sub}, tiles {tiles}")
    _check_group(G, m, _oracle_parts(m, cfgs))
    G.close()


def test_group_merged_subrounds():
    """Merged sub-rounds much smaller than a round: many partition/merge passes
    per round, (key, sketch) pairs of different sketches in one bucket."""
    import torch
    m = sfgen.config_multi(seed=11, n_sketches=40, length_scale=0.03, fat_log2=(8, 12))
    rng = np.random.default_rng(4)
    cfgs = _cfgs(m.w, np.full(m.n, 4), rng.choice([700, 2048, 5000], size=m.n))
    say(f"[case] group merged sub-rounds n={m.n} ops={m.keys.size}")
    G = sf.SketchGroup(cfgs, round_ops=12_000)
    G.update(dev_keys(m.keys), torch.from_numpy(m.ops).cuda(), m.seg)
    sub, tiles = G.rounds()
    say(f"  sub-rounds {sub}, tiles {tiles}")
    lens = np.diff(m.seg.astype(np.int64))
    rounds = int(np.ceil(lens / np.array([c.batch_ops for c in cfgs])).max())
    assert sub > rounds                          # some rounds were split
    ie, de = G.merge_stats()
    assert 0 < ie + de <= m.keys.size
    _check_group(G, m, _oracle_parts(m, cfgs))
    G.close()


def _many_small(n, seed, kb=4):
    """n short mixed streams (120-400 ops over 60 keys each), every sketch one partial tile."""
    rng = np.random.default_rng(seed)
    parts, opss, qs, seg, qseg = [], [], [], [0], [0]
    for i in range(n):
        L = int(rng.integers(120, 400))
        if kb == 4:
            uni = rng.integers(0, 2**32, 60, dtype=np.uint64).astype(np.uint32)
        else:
            uni = rng.integers(0, 256, size=(60, 13), dtype=np.uint8)
        k, o = sfgen.turnstile(uni[rng.zipf(1.2, L) % 60], rng, 0.1)
        parts.append(k)
        opss.append(o)
        qs.append(uni)
        seg.append(seg[-1] + L)
        qseg.append(qseg[-1] + 60)
    return sfgen.MultiWorkload(f"small{n}", 4, 4, rng.choice([64, 128, 256], n), np.concatenate(parts),
                               np.concatenate(opss), np.array(seg, np.uint64), np.concatenate(qs),
                               np.array(qseg, np.uint64))


@pytest.mark.parametrize("kb", [4, 13])
def test_group_more_sketches_than_a_subround_holds(kb):
    """2500 sketches of a few hundred ops: each adds a partial partition tile, so a
    merged sub-round closes on its tile budget (not on ops) and the round splits."""
    import torch
    m = _many_small(2500, seed=21, kb=kb)
    cfgs = _cfgs(m.w, np.full(m.n, 4), np.full(m.n, 4096), kb=kb)
    say(f"[case] group of {m.n} small sketches, {m.keys.shape[0]} ops, key_bytes={kb}")
    G = sf.SketchGroup(cfgs)
    G.update(dev_keys(m.keys), torch.from_numpy(m.ops).cuda(), m.seg)
    sub, tiles = G.rounds()
    say(f"  sub-rounds {sub}, tiles {tiles}")
    assert tiles == m.n and sub >= 2
    _check_group(G, m, _oracle_parts(m, cfgs, kb=kb))
    G.close()


def test_group_replay_and_replan():
    """A repeated call replays the captured graph; new buffers rebuild the plan."""
    import torch
    m = sfgen.config_multi(seed=5, n_sketches=16, length_scale=0.02, fat_log2=(8, 12))
    cfgs = _cfgs(m.w, np.full(m.n, 4), np.full(m.n, 3000))
    refs = _oracle_parts(m, cfgs)
    G = sf.SketchGroup(cfgs)
    keys, ops = dev_keys(m.keys), torch.from_numpy(m.ops).cuda()
    for rep in range(3):
        G.reset()
        G.update(keys, ops, m.seg)
        _check_group(G, m, refs)
    keys2 = keys.clone()                 # same contents, new buffer: plan is rebuilt
    G.reset()
    G.update(keys2, ops, m.seg)
    _check_group(G, m, refs)
    G.close()


def test_group_mixed_rows_and_flow_keys():
    """Different d per sketch (generic row loop) and 13-byte keys."""
    import torch
    rng = np.random.default_rng(9)
    n = 12
    parts, seg, qs, qseg = [], [0], [], [0]
    ops_all = []
    for i in range(n):
        L = int(rng.integers(500, 6000))
        uni = rng.integers(0, 256, size=(max(1, L // 8), 13), dtype=np.uint8)
        ranks = rng.zipf(1.3, L) % uni.shape[0]
        k, o = sfgen.turnstile(uni[ranks], np.random.default_rng(i), 0.1)
        parts.append(k)
        ops_all.append(o)
        seg.append(seg[-1] + L)
        qs.append(uni)
        qseg.append(qseg[-1] + uni.shape[0])
    m = sfgen.MultiWorkload("flows", 0, 4, rng.choice([64, 256, 1000], n), np.concatenate(parts),
                            np.concatenate(ops_all), np.array(seg, np.uint64), np.concatenate(qs),
                            np.array(qseg, np.uint64))
    d = rng.integers(1, 9, n)
    cfgs = _cfgs(m.w, d, rng.choice([333, 4096], n), kb=13, seeds=rng.integers(1, 100, n))
    G = sf.SketchGroup(cfgs)
    assert G.merge_path() == 2                     # rows differ: atomic S1..S5
    G.update(dev_keys(m.keys), torch.from_numpy(m.ops).cuda(), m.seg)
    _check_group(G, m, _oracle_parts(m, cfgs, kb=13))
    G.close()


@pytest.mark.parametrize("graph", [True, False])
def test_group_owner_ranges_split_subrounds(graph):
    """Wide sketches (64 ranges of 2048 cells per row each): a sub-round holds at most 1024
    ranges per row, so rounds split by ranges as well as by ops; the owner path still gives
    every sketch the oracle's state.  Two update calls, the second with other segments."""
    import torch
    m = sfgen.config_multi(seed=5, n_sketches=40, length_scale=0.02, fat_log2=(19, 19))
    cfgs = _cfgs(m.w, np.full(m.n, 4), np.full(m.n, 1 << 14))
    say(f"[case] group owner range cap n={m.n} ops={m.keys.size} graph={graph}")
    G = sf.SketchGroup(cfgs)
    G.set_graph(graph)
    assert G.merge_path() == 1
    seg = m.seg.astype(np.int64)
    lens = np.diff(seg)
    n1 = lens // 2
    # first call: the first half of every stream; second: the rest
    idx1 = np.concatenate([np.arange(seg[i], seg[i] + n1[i]) for i in range(m.n)])
    idx2 = np.concatenate([np.arange(seg[i] + n1[i], seg[i + 1]) for i in range(m.n)])
    seg1 = np.concatenate([[0], np.cumsum(n1)]).astype(np.uint64)
    seg2 = np.concatenate([[0], np.cumsum(lens - n1)]).astype(np.uint64)
    G.update(dev_keys(m.keys[idx1]), torch.from_numpy(m.ops[idx1]).cuda(), seg1)
    sub, tiles = G.rounds()
    say(f"  first call: sub-rounds {sub}, tiles {tiles}")
    assert sub > int(np.ceil(n1 / (1 << 14)).max())     # 40 x 64 ranges > 1024 per sub-round
    G.update(dev_keys(m.keys[idx2]), torch.from_numpy(m.ops[idx2]).cuda(), seg2)
    refs = []
    for i, c in enumerate(cfgs):
        k, o, q = m.part(i)
        n1_i = int(n1[i])
        ref = oracle.Sketch(c.d, c.w, c.z, 4, c.seed_base)
        assert ref.batch(k[:n1_i], o[:n1_i], c.batch_ops, checked=True) == 0
        assert ref.batch(k[n1_i:], o[n1_i:], c.batch_ops, checked=True) == 0
        refs.append((ref.fat(), ref.slim(), ref.query(q)))
    _check_group(G, m, refs)
    G.close()


def test_group_equals_lone_sketches_and_tiles():
    """Group state == one Sketch per stream; tile size does not change it."""
    import torch
    m = sfgen.config_multi(seed=7, n_sketches=10, length_scale=0.05, fat_log2=(10, 12))
    cfgs = _cfgs(m.w, np.full(m.n, 4), np.full(m.n, 4096))
    lone = []
    for i, c in enumerate(cfgs):
        k, o, q = m.part(i)
        s = sf.Sketch(c.d, c.w, c.z, batch_ops=c.batch_ops)
        s.update(dev_keys(k), torch.from_numpy(np.ascontiguousarray(o)).cuda())
        s.sync()
        lone.append((s.export_fat(), s.export_slim(), s.query(dev_keys(q)).cpu().numpy().view(np.uint32)))
        s.close()
    for merge, tile in ((1, 2048), (2, 2048), (0, 256), (0, 2048)):
        G = sf.SketchGroup(cfgs)
        G.set_merge(merge)
        assert G.merge_path() == merge
        G.set_tile(tile)
        G.update(dev_keys(m.keys), torch.from_numpy(m.ops).cuda(), m.seg)
        _check_group(G, m, lone)
        G.close()


def test_group_insert_delete_and_errors():
    import torch
    cfgs = _cfgs([64, 128], [4, 4], [100, 100])
    G = sf.SketchGroup(cfgs)
    keys = torch.arange(0, 300, dtype=torch.int32, device="cuda")
    seg = np.array([0, 100, 300], np.uint64)
    G.insert(keys, seg)
    G.delete(keys, seg)
    G.sync()
    assert not G.export_fat(0).any() and not G.export_fat(1).any()
    assert not G.export_slim(1).any()
    with pytest.raises(sf.SFError):
        G.insert(keys, np.array([0, 200, 100], np.uint64))       # decreasing offsets
    with pytest.raises(sf.SFError):
        G.insert(keys, np.array([0, 100, 1 << 30], np.uint64))   # past the key buffer
    with pytest.raises(sf.SFError):
        G.set_owner_ratio(-1.0)
    with pytest.raises(sf.SFError):
        G.set_merge(3)
    G.close()
    with pytest.raises(sf.SFError):
        sf.SketchGroup([sf.make_config(4, 64, 4, 4), sf.make_config(4, 64, 4, 13)])
