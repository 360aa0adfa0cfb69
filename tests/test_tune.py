"""The batch-size autotuner: its exact counts and error measure on the CPU, and
one tuning run on the GPU (the pick is the fastest candidate within the bound)."""
import numpy as np
import pytest

from paper_1701_04148_amd.tune import are, candidates_for, exact_counts
from tests.oracle_support import random_turnstile


def test_exact_counts_match_a_dictionary_count():
    rng = np.random.default_rng(0)
    for kb in (4, 13):
        keys, ops, uni = random_turnstile(rng, 3000, 200, 0.2, key_bytes=kb)
        absent = (rng.integers(0, 2**32, 50, dtype=np.uint64).astype(np.uint32) if kb == 4
                  else rng.integers(0, 256, size=(50, 13), dtype=np.uint8))
        q = np.concatenate([uni, absent])
        tally = {}
        for k, o in zip(keys, ops):
            kk = bytes(k) if kb == 13 else int(k)
            tally[kk] = tally.get(kk, 0) + (-1 if o == 1 else 1)
        exp = [tally.get(bytes(x) if kb == 13 else int(x), 0) for x in q]
        assert exact_counts(keys, ops, q).tolist() == exp


def test_are_and_saturation():
    f = np.array([0, 1, 2, 100000, 4])
    q = np.array([7, 1, 3, 65535, 4])
    # key 0 (f = 0) ignored; 65535 is exact for f > 65535
    assert are(q, f) == pytest.approx((0 + 0.5 + 0 + 0) / 4)


def test_candidates():
    assert candidates_for(4096, 10**6) == [256 << i for i in range(11)]          # up to 64 w
    assert candidates_for(1 << 20, 1 << 20) == [65536, 131072, 262144, 524288, 1048576]
    assert candidates_for(1 << 20, 10**9) == [65536 << i for i in range(8)]      # up to the cap 2^23
    assert candidates_for(1 << 17, 700_000) == [8192, 16384, 32768, 65536, 131072, 262144, 524288, 1048576]
    assert candidates_for(1 << 12, 100) == [256]


@pytest.mark.gpu
def test_tune_batch_on_gpu():
    import sfgen
    from paper_1701_04148_amd.tune import tune_batch
    w = sfgen.config_small()
    r = tune_batch(w.d, w.w, w.z, w.keys, None, w.queries)
    print(f"[case] tune C1: pick {r.b}, ref {r.ref_b} ARE {r.ref_are:.4f}, bound {r.bound:.4f}, table {r.table}")
    bs = [row[0] for row in r.table]
    assert bs == sorted(bs) and r.ref_b == bs[0]
    feasible = [row for row in r.table if row[3]]
    assert feasible and r.b == min(feasible, key=lambda row: row[2])[0]
    assert all(row[1] <= r.bound for row in feasible)
