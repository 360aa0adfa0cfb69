"""HIP path vs the CPU oracle, element by element, through the C ABI.

Fat counters and query answers are integers and must match bit-exactly; the
Slim must match the oracle's deterministic batch schedule bit-exactly at the
same batch size (and the sequential rule at batch size 1).
"""
import numpy as np
import pytest

import oracle
import paper_1701_04148_amd as sf
import sfgen
from paper_1701_04148_amd.tune import batch_for_width
from tests.gpu_support import assert_same, dev_keys, gpu_run, oracle_run, say
from tests.oracle_support import exact_counts, random_turnstile

pytestmark = pytest.mark.gpu


MERGE_NAMES = {0: "tile", 1: "batch, owner for large batches", 2: "batch+atomic", 3: "batch+owner always"}


def check(d, w, z, kb, keys, ops, queries, b, calls=1, seed_base=1, tag="", merge=0, streams=-1):
    """merge: 0 per-tile merging, 1 batch-wide merge with owner-computes S1..S5 for batches of
    at least w ops where the shape allows, 2 batch-wide merge with atomic S1..S5, 3 owner-computes
    for every batch (sf_set_merge).  streams: the owner path's sf_set_streams mode."""
    say(f"[case] {tag} d={d} w={w} z={z} kb={kb} n={keys.shape[0]} q={queries.shape[0]} "
        f"b={b} calls={calls} merge={MERGE_NAMES[int(merge)]} streams={streams}")
    g = gpu_run(d, w, z, kb, keys, ops, queries, b, seed_base, calls, merge=merge, streams=streams)
    o = oracle_run(d, w, z, kb, keys, ops, queries, b, seed_base, calls)
    assert_same(g[0], o[0], "fat")
    assert_same(g[1], o[1], "slim")
    assert_same(g[2], o[2], "query")
    return g


@pytest.mark.parametrize("d,w,z,kb", [(4, 1024, 4, 4), (1, 64, 4, 4), (3, 1000, 3, 4),
                                      (8, 512, 4, 13), (5, 333, 2, 13), (16, 128, 1, 4),
                                      (2, 4096, 8, 4), (4, 256, 4, 13)])
@pytest.mark.parametrize("b", [1000, 1 << 20])
@pytest.mark.parametrize("merge", [0, 1, 2, 3])
def test_mixed_small(d, w, z, kb, b, merge):
    """Several tiles and a ragged tail: 20011 mixed ops, 30% deletes."""
    rng = np.random.default_rng(d * 7 + w + kb)
    keys, ops, uni = random_turnstile(rng, 20011, 2500, 0.3, key_bytes=kb)
    check(d, w, z, kb, keys, ops, uni, b, tag="mixed_small", merge=merge)


@pytest.mark.parametrize("b", [1, 3, 64])
@pytest.mark.parametrize("merge", [0, 2, 3])
def test_small_batches_and_sequential(b, merge):
    """b = 1 is the sequential SF_F rule of Section 3.5 (the oracle's seq mode)."""
    rng = np.random.default_rng(b)
    keys, ops, uni = random_turnstile(rng, 700, 60, 0.3)
    fat, slim, ans = check(4, 32, 4, 4, keys, ops, uni, b, tag="small_b", merge=merge)
    if b == 1:
        ref = oracle.Sketch(4, 32, 4)
        assert ref.seq(keys, ops, checked=True) == 0
        assert_same(slim, ref.slim(), "slim vs seq")
        assert_same(fat, ref.fat(), "fat vs seq")


@pytest.mark.parametrize("kb", [4, 13])
def test_launch_shape_does_not_change_results(kb):
    """Duplicate merging at tile sizes 256 / 1024 / 2048 ops gives identical state."""
    import torch
    wl = sfgen.make("tiles", d=4, w=2048, z=4, n_universe=5000, n_ops=200_000, s=1.3, p_del=0.15,
                    key_bytes=kb, seed=11)
    ref = oracle_run(4, 2048, 4, kb, wl.keys, wl.ops, wl.universe, 50_000)
    for tile in (256, 1024, 2048):
        say(f"[case] tile={tile} kb={kb}")
        sk = sf.Sketch(4, 2048, 4, key_bytes=kb, batch_ops=50_000)
        sk.set_tile(tile)
        sk.update(dev_keys(wl.keys), torch.from_numpy(wl.ops).cuda())
        q = sk.query(dev_keys(wl.universe)).cpu().numpy().view(np.uint32)
        sk.sync()
        assert_same(sk.export_fat(), ref[0], f"fat tile={tile}")
        assert_same(sk.export_slim(), ref[1], f"slim tile={tile}")
        assert_same(q, ref[2], f"query tile={tile}")
        sk.close()


def test_several_calls_start_new_batches():
    """Every update call starts a new schedule batch."""
    rng = np.random.default_rng(5)
    keys, ops, uni = random_turnstile(rng, 30000, 3000, 0.2)
    check(4, 512, 4, 4, keys, ops, uni, 4096, calls=7, tag="calls")


def test_insert_and_delete_entry_points():
    """sf_insert / sf_delete (uniform op) equal sf_update with the same ops."""
    import torch
    rng = np.random.default_rng(8)
    keys, ops, uni = random_turnstile(rng, 5000, 400, 0.0)
    dels = keys[rng.permutation(keys.size)[:1500]]
    sk = sf.Sketch(4, 256, 4, batch_ops=2048)
    sk.insert(dev_keys(keys))
    sk.delete(dev_keys(dels))
    q = sk.query(dev_keys(uni)).cpu().numpy().view(np.uint32)
    sk.sync()
    ref = oracle.Sketch(4, 256, 4)
    assert ref.batch(keys, None, 2048, True) == 0
    assert ref.batch(dels, np.ones(dels.size, np.uint8), 2048, True) == 0
    assert_same(sk.export_fat(), ref.fat(), "fat")
    assert_same(sk.export_slim(), ref.slim(), "slim")
    assert_same(q, ref.query(uni), "query")
    sk.close()


@pytest.mark.parametrize("merge", [0, 1, 2])
def test_small_config_full_size(merge):
    """1M Zipf(1.0) inserts over 100K keys, d=4, Fat 4x65536, Slim 4x16384; all 100K queried."""
    wl = sfgen.config_small()
    fat, slim, ans = check(wl.d, wl.w, wl.z, 4, wl.keys, None, wl.queries, 65536, tag="c1", merge=merge)
    f = exact_counts(wl.keys, None, wl.queries)
    assert (ans.astype(np.int64) >= np.minimum(f, 65535)).all()


@pytest.mark.parametrize("skew,merge", [(1.4, 0), (1.4, 1), (0.6, 1), (1.0, 1), (1.0, 2)])
def test_main_config_scaled(skew, merge):
    """The 32M-op configuration divided by 8 (4M ops, 10% deletes, w=2^17)."""
    wl = sfgen.config_main(skew, scale=8)
    check(wl.d, wl.w, wl.z, 4, wl.keys, wl.ops, wl.queries, 1 << 18, tag="c2/8", merge=merge)
    if merge == 1:   # per call four batches of 5 * 2^16 ops (>= w = 2^17: owner) and a tail of 23K (atomic)
        check(wl.d, wl.w, wl.z, 4, wl.keys, wl.ops, wl.queries, 5 << 16, calls=3, tag="c2/8 mixed paths",
              merge=1)


@pytest.mark.parametrize("d,w,z,kb,b,calls", [(4, 1024, 4, 4, 1024, 1), (3, 1000, 3, 4, 1500, 3),
                                               (8, 512, 4, 13, 600, 2), (4, 1 << 14, 4, 4, 1 << 14, 4),
                                               (5, 333, 2, 13, 333, 1)])
@pytest.mark.parametrize("merge", [1, 3])
def test_owner_two_streams(d, w, z, kb, b, calls, merge):
    """The owner path with the next batch's partition, merge and pairs on a second stream:
    many batches per call (so the two sides overlap and the sets of pairs and column starts
    rotate), several calls, ragged tails that take the atomic path in mode 1."""
    rng = np.random.default_rng(d * 13 + w + b)
    keys, ops, uni = random_turnstile(rng, 40011, 4000, 0.25, key_bytes=kb)
    check(d, w, z, kb, keys, ops, uni, b, calls=calls, tag="two streams", merge=merge, streams=1)


@pytest.mark.parametrize("d,w,z,kb", [(4, 1 << 14, 4, 4), (3, 1000, 3, 13), (8, 4096, 2, 4)])
def test_owner_range_sizes(d, w, z, kb):
    """Every range size the owner path accepts for the shape (from 16 cells, or the smallest
    that keeps a row within its range limit, up to 8192 Fat counters per range) gives the
    oracle's state; ranges larger than the row (one ragged range) included."""
    import torch
    rng = np.random.default_rng(d * 5 + w)
    keys, ops, uni = random_turnstile(rng, 60_000, 6000, 0.2, key_bytes=kb)
    b = 1 << 14
    o = oracle_run(d, w, z, kb, keys, ops, uni, b, 1, 2)
    sk = sf.Sketch(d, w, z, key_bytes=kb, batch_ops=b)
    from paper_1701_04148_amd.tune import owner_shifts
    shifts = owner_shifts(sk)
    default = sk.owner_range()
    say(f"[case] owner range sizes d={d} w={w} z={z} kb={kb}: shifts {shifts}, default {default}")
    assert shifts == list(range(shifts[0], shifts[-1] + 1))
    assert shifts[0] <= default <= shifts[-1]
    assert (1 << shifts[-1]) * z <= 8192
    with pytest.raises(sf.SFError):
        sk.set_owner_range(shifts[-1] + 1)
    with pytest.raises(sf.SFError):
        sk.set_owner_range(shifts[0] - 1)
    sk.close()
    for shift in shifts:
        g = gpu_run(d, w, z, kb, keys, ops, uni, b, 1, 2, merge=3, shift=shift)
        assert_same(g[0], o[0], f"fat shift={shift}")
        assert_same(g[1], o[1], f"slim shift={shift}")
        assert_same(g[2], o[2], f"query shift={shift}")


def test_owner_two_streams_uniform_ops():
    """Insert-only then delete-only calls (no k_level in a delete batch) on two streams."""
    import torch
    rng = np.random.default_rng(21)
    keys, _, uni = random_turnstile(rng, 30000, 3000, 0.0)
    dels = keys[rng.permutation(keys.size)[:9000]]
    say("[case] two streams, insert then delete calls")
    sk = sf.Sketch(4, 1024, 4, batch_ops=2048)
    sk.set_merge(3)
    with pytest.raises(sf.SFError):
        sk.set_streams(2)
    sk.set_streams(1)
    sk.insert(dev_keys(keys))
    sk.delete(dev_keys(dels))
    sk.insert(dev_keys(keys[:5000]))
    q = sk.query(dev_keys(uni)).cpu().numpy().view(np.uint32)
    sk.sync()
    ref = oracle.Sketch(4, 1024, 4)
    assert ref.batch(keys, None, 2048, True) == 0
    assert ref.batch(dels, np.ones(dels.size, np.uint8), 2048, True) == 0
    assert ref.batch(keys[:5000], None, 2048, True) == 0
    assert_same(sk.export_fat(), ref.fat(), "fat")
    assert_same(sk.export_slim(), ref.slim(), "slim")
    assert_same(q, ref.query(uni), "query")
    sk.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("skew", [0.6, 1.0, 1.4])
def test_main_config_full_size_as_benchmarked(skew):
    """The 32M-op configuration at full size (w=2^20, 10% deletes) at every skew, with
    the benchmark's schedule batch 2^23 and launch settings: Fat, Slim and all 2M
    answers bit-exact against the oracle."""
    wl = sfgen.config_main(skew)
    check(wl.d, wl.w, wl.z, 4, wl.keys, wl.ops, wl.queries, batch_for_width(wl.w),
          tag=f"c2 full s={skew}", merge=1)
    if skew == 1.0:   # the same with the partition side on a second stream
        check(wl.d, wl.w, wl.z, 4, wl.keys, wl.ops, wl.queries, batch_for_width(wl.w),
              tag=f"c2 full s={skew}", merge=1, streams=1)


@pytest.mark.parametrize("merge", [0, 1, 2])
def test_flow_config_scaled(merge):
    """13-byte flow keys, d=8, divided by 64 (2M packets over 62.5K flows)."""
    wl = sfgen.config_flows(scale=64)
    check(wl.d, wl.w, wl.z, 13, wl.keys, None, wl.queries, 1 << 18, tag="c3/64", merge=merge)


def test_batch_merge_with_one_hot_key():
    """One key is 60% of a 2^20-op batch (one bucket far larger than a merge chunk)."""
    rng = np.random.default_rng(4)
    n = 1 << 20
    keys = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    keys[rng.random(n) < 0.6] = 12345
    ops = np.zeros(n, np.uint8)
    q = np.unique(keys)[:50_000]
    check(4, 1 << 14, 4, 4, keys, ops, q, n, tag="hot", merge=1)
    check(4, 1 << 14, 4, 4, keys, ops, q, n, tag="hot", merge=2)
    check(4, 1 << 14, 4, 4, keys, ops, q, 1 << 12, tag="hot, small batches", merge=3)


@pytest.mark.parametrize("kb", [4, 13])
def test_merge_chunk_packing_shapes(kb):
    """One batch whose bucket sizes are built around the rule that packs small
    buckets into shared merge chunks: empty, tiny, exactly half a chunk, one
    key over half, one chunk, several chunks, runs of small buckets across
    half-chunk windows and next to big ones, in both op types.  Keys are
    picked by their row-0 column, which decides a lone sketch's bucket."""
    K = 8192 if kb == 4 else 2048                 # keys per merge chunk of a lone sketch
    d, w, z, nb = 4, 1 << 14, 4, 32
    H = K // 2
    ins = [0, 3, H, H + 1, 5, 5 * H, 7, 0, K // 4, K // 4, K // 4, K // 4 + 3, 1, 1, 1, 6 * H,
           H, H, 0, 0, 10, K - 1, K, K + 1, 2, 0, K // 3, K // 3, K // 3, 4, 0, 100]
    dels = [0, 3, 1, H, 0, H + 1, 7, 0, 2, 0, K // 4, 1, 1, 0, 1, 3 * H,
            0, H, 0, 0, 10, 5, K, 9, 2, 0, 1, 0, K // 3, 4, 0, 100]
    n = sum(ins) + sum(dels)
    assert nb // 2 * K < n <= nb * K               # so that the batch gets exactly nb buckets per op type
    rng = np.random.default_rng(70 + kb)
    if kb == 4:
        cand = rng.choice(2**32, size=160_000, replace=False).astype(np.uint32)
    else:
        cand = rng.integers(0, 256, size=(160_000, 13), dtype=np.uint8)
    h, _ = oracle.Sketch(d, w, z, kb).indices(cand)
    bucket = h[:, 0].astype(np.int64) * nb // w
    ins_keys, del_keys = [], []
    for j in range(nb):
        pool = cand[bucket == j]
        if ins[j] == 0:
            continue
        distinct = pool[: max(1, ins[j] // 3)]
        occ = distinct[rng.integers(0, distinct.shape[0], ins[j]) % distinct.shape[0]]
        ins_keys.append(occ)
        if dels[j]:
            del_keys.append(occ[rng.permutation(ins[j])[: dels[j]]])   # deletes of inserted copies
    ki = np.concatenate(ins_keys)
    kd = np.concatenate(del_keys)
    ki = ki[rng.permutation(ki.shape[0])]
    kd = kd[rng.permutation(kd.shape[0])]
    keys = np.concatenate([ki, kd])
    ops = np.concatenate([np.zeros(ki.shape[0], np.uint8), np.ones(kd.shape[0], np.uint8)])
    q = np.concatenate([np.unique(ki, axis=0), cand[-1000:]])
    for mode in (1, 2):
        check(d, w, z, kb, keys, ops, q, 1 << 20, tag="packing", merge=mode)


def test_query_exported_slim_collector():
    """The collector answers from the exported uint16 Slim alone (sf_query_slim)."""
    import torch
    rng = np.random.default_rng(3)
    for kb in (4, 13):
        keys, ops, uni = random_turnstile(rng, 8000, 900, 0.2, key_bytes=kb)
        sk = sf.Sketch(4, 512, 4, key_bytes=kb, batch_ops=4096)
        sk.update(dev_keys(keys), torch.from_numpy(ops).cuda())
        direct = sk.query(dev_keys(uni)).cpu().numpy()
        slim = torch.from_numpy(sk.export_slim().astype(np.uint16).view(np.int16)).cuda()
        out = torch.empty(uni.shape[0], dtype=torch.int32, device="cuda")
        sf.sf_query_slim(slim, sk.cfg, dev_keys(uni), out)
        torch.cuda.synchronize()
        assert_same(out.cpu().numpy(), direct, "collector query")
        exp = oracle.query_slim(sk.export_slim(), 4, 512, 4, uni, key_bytes=kb)
        assert_same(out.cpu().numpy().view(np.uint32), exp, "collector vs oracle")
        sk.close()


@pytest.mark.parametrize("d,w,z,kb,nq", [(4, 1 << 20, 4, 4, 300_000), (8, 1 << 19, 1, 4, 2_500_000),
                                         (2, 1 << 21, 2, 13, 200_000)])
def test_query_one_row_per_xcd(d, w, z, kb, nq):
    """After an export a Slim larger than 4 MiB is queried one row per XCD (per-row
    counters in scratch, then a minimum pass), in runs that fit the scratch
    (three runs for the d=8, z=1 case).  Answers equal the records path's and
    the oracle's query on the exported Slim."""
    import torch
    rng = np.random.default_rng(d * 31 + kb)
    keys, ops, uni = random_turnstile(rng, 400_000, 60_000, 0.1, key_bytes=kb)
    if kb == 4:
        extra = rng.integers(0, 2**32, nq - uni.shape[0], dtype=np.uint64).astype(np.uint32)
    else:
        extra = rng.integers(0, 256, size=(nq - uni.shape[0], 13), dtype=np.uint8)
    q = np.concatenate([uni, extra])
    say(f"[case] row-per-XCD query d={d} w={w} z={z} kb={kb} q={nq}")
    sk = sf.Sketch(d, w, z, key_bytes=kb, batch_ops=1 << 18)
    sk.update(dev_keys(keys), torch.from_numpy(ops).cuda())
    dq = dev_keys(q)
    before = sk.query(dq).cpu().numpy().view(np.uint32).copy()      # records path
    slim = sk.export_slim()
    after = sk.query(dq).cpu().numpy().view(np.uint32)               # dense copy, one row per XCD
    sk.close()
    assert_same(after, before, "row-per-XCD query vs records query")
    sample = np.concatenate([np.arange(min(nq, 150_000)), rng.integers(0, nq, 20_000)])
    exp = oracle.query_slim(slim, d, w, z, q[sample], key_bytes=kb)
    assert_same(after[sample], exp, "row-per-XCD query vs oracle on the exported Slim")


def test_query_reads_exported_copy_only_while_fresh():
    """sf_query answers from the sketch's dense copy made by sf_export_slim until
    the next update or reset: before export, after export, after more updates
    (stale copy must not be used), after reset -- all equal to the oracle."""
    import torch
    rng = np.random.default_rng(17)
    keys, ops, uni = random_turnstile(rng, 30_000, 3000, 0.15)
    half = keys.shape[0] // 2
    ref = oracle.Sketch(4, 1024, 4)
    sk = sf.Sketch(4, 1024, 4, batch_ops=5000)
    dev16 = torch.empty(4 * 1024, dtype=torch.int16, device="cuda")
    for lo, hi in ((0, half), (half, keys.shape[0])):
        sk.update(dev_keys(keys[lo:hi]), torch.from_numpy(ops[lo:hi]).cuda())
        assert ref.batch(keys[lo:hi], ops[lo:hi], 5000, checked=True) == 0
        exp = ref.query(uni)
        assert_same(sk.query(dev_keys(uni)).cpu().numpy().view(np.uint32), exp, "query before export")
        sf.sf_export_slim(sk._h, dev16)                     # device destination
        assert_same(dev16.cpu().numpy().view(np.uint16).reshape(4, 1024), ref.slim(), "exported Slim")
        assert_same(sk.query(dev_keys(uni)).cpu().numpy().view(np.uint32), exp, "query after export")
        assert_same(sk.export_slim(), ref.slim(), "second export (host destination)")
    sk.reset()
    assert not sk.query(dev_keys(uni)).cpu().numpy().any()
    sk.close()


def test_device_export_is_stream_ordered():
    """A device-destination sf_export_slim returns without waiting for its kernel;
    work queued after it on the same stream -- sf_query_slim reading the exported
    buffer, then another update and export into that buffer -- sees its result.
    w = 2^20 so that the export (4M cells) is still running when the call returns."""
    import torch
    d, w, z, b = 4, 1 << 20, 4, 1 << 17
    rng = np.random.default_rng(23)
    keys, ops, uni = random_turnstile(rng, 300_000, 40_000, 0.1)
    half = keys.shape[0] // 2
    ref = oracle.Sketch(d, w, z)
    sk = sf.Sketch(d, w, z, batch_ops=b)
    dev16 = torch.empty(d * w, dtype=torch.int16, device="cuda")
    q = dev_keys(uni)
    out = torch.empty(uni.shape[0], dtype=torch.int32, device="cuda")
    for lo, hi in ((0, half), (half, keys.shape[0])):
        sk.update(dev_keys(keys[lo:hi]), torch.from_numpy(ops[lo:hi]).cuda())
        sf.sf_export_slim(sk._h, dev16)           # ordered on the sketch's (null) stream
        sf.sf_query_slim(dev16, sk.cfg, q, out)   # the same stream: reads the finished copy
        assert ref.batch(keys[lo:hi], ops[lo:hi], b, checked=True) == 0
        assert_same(out.cpu().numpy().view(np.uint32), ref.query(uni), "query of the exported copy")
        assert_same(dev16.cpu().numpy().view(np.uint16).reshape(d, w), ref.slim(), "exported Slim")
    sk.close()


def test_empty_and_tiny_inputs():
    import torch
    sk = sf.Sketch(4, 64, 4, batch_ops=8)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    sk.insert(e)
    sk.delete(e)
    sk.update(e, torch.empty(0, dtype=torch.uint8, device="cuda"))
    assert sk.query(e).numel() == 0
    one = torch.tensor([42], dtype=torch.int32, device="cuda")
    sk.insert(one)
    assert int(sk.query(one).item()) == 1
    sk.delete(one)
    assert int(sk.query(one).item()) == 0
    assert not sk.export_fat().any() and not sk.export_slim().any()
    sk.close()


def test_saturation_on_gpu():
    """Slim saturates at 65535 while the Fat keeps the exact count."""
    import torch
    k = torch.full((70000,), 7, dtype=torch.int32, device="cuda")
    sk = sf.Sketch(4, 64, 4, batch_ops=1 << 16)
    sk.insert(k)
    assert int(sk.query(k[:1]).item()) == 65535
    assert sk.export_fat().max() == 70000
    sk.delete(k[:10000])
    assert int(sk.query(k[:1]).item()) == 60000
    sk.close()


def test_bad_arguments_rejected_without_launch():
    import torch
    sk = sf.Sketch(4, 64, 4, batch_ops=8)
    buf = torch.zeros(16, dtype=torch.int32, device="cuda")
    mis = buf.view(torch.uint8)[1:9]
    assert sf.lib().sf_insert(sk._h, mis.data_ptr(), 2) == sf.SF_EINVAL      # misaligned
    assert sf.lib().sf_insert(sk._h, buf.data_ptr(), 1 << 26) == sf.SF_EINVAL  # past the buffer
    import numpy as _np
    host = _np.zeros(16, _np.int32)
    assert sf.lib().sf_insert(sk._h, host.ctypes.data, 16) == sf.SF_EINVAL   # pageable host
    small = _np.zeros(3, _np.uint16)
    assert sf.lib().sf_export_slim(sk._h, small.ctypes.data, 3) == sf.SF_EINVAL
    sk.close()
    assert sf.lib().sf_sync(sk._h or None) == sf.SF_ESTATE


def test_hbm_budget_admission():
    c = sf.make_config(4, 1 << 16, 4, 4, 1, 1 << 16)
    with pytest.raises(sf.SFError) as e:
        sf.sf_create(c, sf.sf_footprint(c) - 1)
    assert e.value.status == sf.SF_ENOMEM
    h = sf.sf_create(c, sf.sf_footprint(c))
    sf.sf_destroy(h)


@pytest.mark.timeout(900)
def test_flow_config_full_size_bit_exact():
    """128M 13-byte packets, d=8, Fat 8x2^23, Slim 8x2^21, in the launch shape the
    benchmark uses: Fat, Slim and all 16M answers bit-exact against the oracle's batch
    schedule at the same b (the oracle runs in a thread while the GPU works).  Also the
    paper's invariants: every Slim cell is at most min(65535, its bucket max)
    (Appendix I); every flow's answer is at least min(f, 65535) (Appendix II)."""
    import threading
    wl = sfgen.config_flows()
    b = batch_for_width(wl.w)
    counts = wl.meta["universe_counts"]
    say(f"[case] flows full size: {wl.n_ops} packets, {wl.n_queries} queries, b={b}")
    ref = {}

    def run_oracle():
        ref["fat"], ref["slim"], ref["q"] = oracle_run(wl.d, wl.w, wl.z, 13, wl.keys, None, wl.queries, b)

    th = threading.Thread(target=run_oracle)
    th.start()
    try:
        sk = sf.Sketch(wl.d, wl.w, wl.z, key_bytes=13, batch_ops=b)
        assert sk.merge_path() == 1                  # owner-computes S1..S5, as benchmarked
        sk.insert(dev_keys(wl.keys))
        ans = sk.query(dev_keys(wl.queries)).cpu().numpy().view(np.uint32)
        sk.sync()
        fat, slim = sk.export_fat(), sk.export_slim()
        sk.close()
    finally:
        th.join()
    say("[case] flows full size: oracle done")
    assert_same(fat, ref["fat"], "fat")
    assert_same(slim, ref["slim"], "slim")
    assert_same(ans, ref["q"], "query")
    bmax = fat.max(axis=2)
    assert (slim.astype(np.int64) <= np.minimum(bmax, 65535)).all()
    f = np.zeros(wl.n_queries, np.int64)
    f[:counts.size] = counts                       # queries = the flows, then absent keys
    assert (ans.astype(np.int64) >= np.minimum(f, 65535)).all()


def test_host_fed_updates_equal_device_updates():
    """sf_update_host (pinned host keys, chunked copies overlapping the updates)
    reaches exactly the state of sf_update on device buffers and of the oracle's
    batch schedule over the same calls; two calls in a row
    reuse the chunk buffers; pageable memory and bad chunk sizes are refused."""
    import torch
    wl = sfgen.config_main(1.0, scale=64)                     # 500K ops, w = 2^14
    b = 1 << 14
    n = wl.keys.shape[0]
    ref = sf.Sketch(wl.d, wl.w, wl.z, batch_ops=b)
    ref.update(dev_keys(wl.keys), torch.from_numpy(wl.ops).cuda())
    ref.sync()
    say(f"[case] host-fed updates n={n} b={b}")
    hk = torch.from_numpy(wl.keys.view(np.int32)).pin_memory()
    ho = torch.from_numpy(wl.ops).pin_memory()
    sk = sf.Sketch(wl.d, wl.w, wl.z, batch_ops=b)
    half = (n // 2) // b * b                                  # split at a batch boundary
    sk.update_host(hk[:half], ho[:half], chunk_ops=3 * b)
    sk.update_host(hk[half:], ho[half:], chunk_ops=3 * b)
    sk.sync()
    assert_same(sk.export_fat(), ref.export_fat(), "fat")
    assert_same(sk.export_slim(), ref.export_slim(), "slim")
    q = dev_keys(wl.queries)
    got_q = sk.query(q).cpu().numpy().view(np.uint32)
    assert_same(got_q, ref.query(q).cpu().numpy().view(np.uint32), "queries")
    # and against the oracle's batch schedule over the same two calls
    orc = oracle.Sketch(wl.d, wl.w, wl.z)
    assert orc.batch(wl.keys[:half], wl.ops[:half], b, checked=True) == 0
    assert orc.batch(wl.keys[half:], wl.ops[half:], b, checked=True) == 0
    assert_same(sk.export_fat(), orc.fat(), "fat vs oracle")
    assert_same(sk.export_slim(), orc.slim(), "slim vs oracle")
    assert_same(got_q, orc.query(wl.queries), "queries vs oracle")
    ins = sf.Sketch(wl.d, wl.w, wl.z, batch_ops=b)             # insert-only form (ops = None)
    ins.update_host(hk[:half], None, chunk_ops=b)
    ref2 = sf.Sketch(wl.d, wl.w, wl.z, batch_ops=b)
    ref2.insert(dev_keys(wl.keys[:half]))
    ins.sync()
    ref2.sync()
    assert_same(ins.export_fat(), ref2.export_fat(), "fat, inserts")
    orc2 = oracle.Sketch(wl.d, wl.w, wl.z)
    assert orc2.batch(wl.keys[:half], None, b, checked=True) == 0
    assert_same(ins.export_fat(), orc2.fat(), "fat, inserts vs oracle")
    assert_same(ins.export_slim(), orc2.slim(), "slim, inserts vs oracle")
    rc = sf.lib().sf_update_host(sk._h, wl.keys.ctypes.data, None, 1000, b)   # pageable numpy memory
    assert rc == sf.SF_EINVAL
    rc = sf.lib().sf_update_host(sk._h, hk.data_ptr(), None, 1000, b + 1)     # not a multiple of b
    assert rc == sf.SF_EINVAL
    for s_ in (sk, ref, ins, ref2):
        s_.close()


def test_host_fed_query_pipeline():
    """sf_query_host (pinned host keys split over n streams, the first n_keys mod n
    streams taking one key more, each copying in, querying and copying out) answers
    exactly as sf_query and the oracle, with the Slim's dense copy fresh or not, for
    stream counts that do not divide the key count; later updates wait for it; bad
    arguments are refused."""
    import torch
    wl = sfgen.config_main(1.0, scale=64)                     # 500K ops, w = 2^14
    b = 1 << 15
    half = wl.n_ops // 2
    sk = sf.Sketch(wl.d, wl.w, wl.z, batch_ops=b)
    orc = oracle.Sketch(wl.d, wl.w, wl.z)
    sk.update(dev_keys(wl.keys[:half]), torch.from_numpy(wl.ops[:half]).cuda())
    assert orc.batch(wl.keys[:half], wl.ops[:half], b, checked=True) == 0
    q = wl.queries[:100_003]
    hq = torch.from_numpy(q.view(np.int32)).pin_memory()
    ref = orc.query(q)
    for streams in (1, 3, 4, 16):
        say(f"[case] query pipeline streams={streams} n={q.shape[0]} (records)")
        got = sk.query_host(hq, streams=streams).numpy().view(np.uint32)
        assert_same(got, ref, f"host-fed query, {streams} streams")
    sf.sf_export_slim(sk._h, torch.empty(wl.d * wl.w, dtype=torch.int16, device="cuda"))
    for streams in (2, 7):
        say(f"[case] query pipeline streams={streams} (dense copy)")
        got = sk.query_host(hq, streams=streams).numpy().view(np.uint32)
        assert_same(got, ref, f"host-fed query on the dense copy, {streams} streams")
    tiny = torch.from_numpy(q[:5].view(np.int32)).pin_memory()  # fewer keys than streams
    assert_same(sk.query_host(tiny, streams=16).numpy().view(np.uint32), ref[:5], "5 keys, 16 streams")
    # the second half of the stream after the pipelined queries, then queries again
    sk.update(dev_keys(wl.keys[half:]), torch.from_numpy(wl.ops[half:]).cuda())
    assert orc.batch(wl.keys[half:], wl.ops[half:], b, checked=True) == 0
    got = sk.query_host(hq, streams=4).numpy().view(np.uint32)
    assert_same(got, orc.query(q), "after a later update")
    assert_same(sk.query(dev_keys(q)).cpu().numpy().view(np.uint32), got, "device query")
    out = torch.empty(q.shape[0], dtype=torch.int32).pin_memory()
    assert sf.lib().sf_query_host(sk._h, q.ctypes.data, q.shape[0], out.data_ptr(), 4) == sf.SF_EINVAL
    assert sf.lib().sf_query_host(sk._h, hq.data_ptr(), q.shape[0], out.data_ptr(), 0) == sf.SF_EINVAL
    assert sf.lib().sf_query_host(sk._h, hq.data_ptr(), q.shape[0], out.data_ptr(), 17) == sf.SF_EINVAL
    sk.close()
