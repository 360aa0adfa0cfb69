"""sf_query_slim_noalloc (the entry point for callers that cannot allocate)
against sf_query_slim through the C ABI: two calls in a row, the second with
a smaller input, bit-exact; and the oracle's collector query over the same
exported Slim.  Both the one-row-per-XCD path (Slim > 4 MiB, d dividing 8)
and the one-pass path are covered, and an oversized request is refused."""
import numpy as np
import pytest

import oracle
import paper_1701_04148_amd as sf
import sfgen
from gpu_support import assert_same, dev_keys, say

pytestmark = pytest.mark.gpu


def _exported(d, w, z, kb, keys):
    import torch
    sk = sf.Sketch(d, w, z, key_bytes=kb, batch_ops=1 << 18)
    sk.insert(dev_keys(keys))
    slim = torch.empty(d * w, dtype=torch.int16, device="cuda")
    sf.sf_export_slim(sk._h, slim)
    cfg = sk.cfg
    sk.close()
    return slim, cfg


def _both(slim, cfg, q):
    import torch
    n = q.shape[0]
    a = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    b = torch.full((n,), -2, dtype=torch.int32, device="cuda")
    sf.sf_query_slim(slim, cfg, dev_keys(q), a)
    sf.sf_query_slim_noalloc(slim, cfg, dev_keys(q), b)
    torch.cuda.synchronize()
    return a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("d,w,z,kb,n1,n2", [
    (4, 1 << 20, 4, 4, 1_500_000, 300_001),   # 8 MiB Slim: one row per XCD, n*d near the limit
    (8, 1 << 19, 4, 13, 900_000, 77_777),     # 8 MiB Slim, 13-byte keys, d = 8
    (3, 4096, 4, 4, 200_000, 999),            # small Slim, d not dividing 8: one pass
])
def test_noalloc_query_equals_allocating_query(d, w, z, kb, n1, n2):
    rng = np.random.default_rng(d * 1000 + kb)
    if kb == 4:
        keys = rng.integers(0, 1 << 32, size=400_000, dtype=np.uint64).astype(np.uint32)
        q1 = np.concatenate([keys[:n1 // 2], rng.integers(0, 1 << 32, size=n1 - n1 // 2,
                                                            dtype=np.uint64).astype(np.uint32)])
        q2 = rng.integers(0, 1 << 32, size=n2, dtype=np.uint64).astype(np.uint32)
        q2[: n2 // 3] = keys[: n2 // 3]
    else:
        keys = rng.integers(0, 256, size=(400_000, 13), dtype=np.uint8)
        q1 = np.concatenate([keys[:n1 // 2], rng.integers(0, 256, size=(n1 - n1 // 2, 13), dtype=np.uint8)])
        q2 = rng.integers(0, 256, size=(n2, 13), dtype=np.uint8)
        q2[: n2 // 3] = keys[: n2 // 3]
    # a skewed insert stream so that answers spread over many values
    zipf = sfgen.zipf_ranks(np.random.default_rng(7), keys.shape[0], 1.1, 3_000_000)
    stream = keys[zipf]
    say(f"[case] noalloc d={d} w={w} kb={kb} n1={n1} n2={n2}")
    slim, cfg = _exported(d, w, z, kb, stream)
    host_slim = slim.cpu().numpy().view(np.uint16).reshape(d, w)
    for q in (q1, q2):                         # two calls in a row, the second smaller
        a, b = _both(slim, cfg, q)
        assert_same(b, a, "noalloc vs sf_query_slim")
        assert_same(b, oracle.query_slim(host_slim, d, w, z, q, kb), "noalloc vs oracle")
        assert (b != 0).any()


def test_noalloc_query_rejects_more_than_its_scratch():
    import torch
    d, w = 4, 1 << 20
    cfg = sf.make_config(d, w, 4)
    slim = torch.zeros(d * w, dtype=torch.int16, device="cuda")
    n = sf.NOALLOC_QUERY_COUNTERS // d + 1
    keys = torch.zeros(n, dtype=torch.int32, device="cuda")
    out = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(sf.SFError) as e:
        sf.sf_query_slim_noalloc(slim, cfg, keys, out)
    assert e.value.status == sf.SF_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert (out == 7).all()                    # nothing ran
    sf.sf_query_slim_noalloc(slim, cfg, keys[:-1], out)   # at the limit it runs
    torch.cuda.synchronize()
    assert (out[:-1] == 0).all()
