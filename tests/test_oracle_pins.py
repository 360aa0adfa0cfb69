"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test names the property and where it comes from.  None of them re-types
the oracle's formulas: expected values come from scikit-learn's hash, from
brute-force histograms and counts, from the paper's worked example, from
closed forms that hold in special cases, or from a second transcription.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import sfpy
from tests.oracle_support import (exact_counts, histogram_fat, random_turnstile, sk_hash,
                                  sk_indices)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SLIM_MAX = 65535


# ---------------------------------------------------------------- hashing

def test_murmur3_matches_sklearn():
    """Hash contract: MurmurHash3_x86_32 (checked against scikit-learn)."""
    from sklearn.utils import murmurhash3_32
    rng = np.random.default_rng(7)
    for length in range(0, 33):
        for _ in range(25):
            data = rng.integers(0, 256, length, dtype=np.uint8).tobytes()
            seed = int(rng.integers(0, 2**32))
            assert oracle.murmur3_32(data, seed) == murmurhash3_32(data, seed=seed, positive=True)


@pytest.mark.parametrize("d,w,z,kb", [(4, 16384, 4, 4), (3, 40000, 3, 4), (8, 1024, 4, 13),
                                      (5, 7, 5, 13), (2, 2**16, 2**16, 4)])
def test_index_split_eq1(d, w, z, kb):
    """Eq. (1), 0-based: c = g mod wz, h = c mod w, f = c div w (incl. non powers of 2)."""
    rng = np.random.default_rng(d * 1000 + w)
    keys = (rng.integers(0, 2**32, 3000, dtype=np.uint64).astype(np.uint32) if kb == 4
            else rng.integers(0, 256, (3000, 13), dtype=np.uint8))
    h, f = oracle.Sketch(d, w, z, kb).indices(keys)
    eh, ef = sk_indices(keys, d, w, z)
    np.testing.assert_array_equal(h, eh)
    np.testing.assert_array_equal(f, ef)
    assert h.max() < w and f.max() < z


# ---------------------------------------------------------------- P1, P2: Fat

@pytest.mark.parametrize("mode,b", [("seq", 0), ("batch", 1), ("batch", 7), ("batch", 256),
                                    ("batch", 10**9)])
@pytest.mark.parametrize("kb", [4, 13])
def test_fat_is_histogram(mode, b, kb):
    """The Fat-subsketch is a CM-sketch over w*z columns per row (Sections 3.1, 3.4):
    after any stream its counters are the signed histogram of the row columns, in
    every update mode.  Row sums equal net stream weight (inserts - deletes)."""
    rng = np.random.default_rng(11 + kb)
    keys, ops, _ = random_turnstile(rng, 4000, 300, 0.3, key_bytes=kb)
    d, w, z = 3, 64, 4
    sk = oracle.Sketch(d, w, z, kb)
    rc = sk.seq(keys, ops, checked=True) if mode == "seq" else sk.batch(keys, ops, b, checked=True)
    assert rc == 0
    h, f = sk_indices(keys, d, w, z)
    fat = sk.fat()
    np.testing.assert_array_equal(fat, histogram_fat(h, f, ops, d, w, z))
    net = int((ops == 0).sum() - (ops == 1).sum())
    assert all(int(fat[i].astype(np.int64).sum()) == net for i in range(d))
    np.testing.assert_array_equal(sk.fat_histogram(keys, ops), fat)


# ---------------------------------------------------------------- P3: paper example

def _example():
    with open(os.path.join(GOLDEN, "paper_deletion_example.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("mode", ["seq", "batch1"])
@pytest.mark.parametrize("z,slots", [(1, ([0, 0], [0, 0])), (2, ([0, 0], [1, 1]))])
def test_paper_deletion_example(mode, z, slots):
    """Section 3.2, Figure 3: after inserting e1 and e2 the Slim is A1=[1,0], A2=[1,1]
    (printed by the paper).  Deleting e1 naively would answer q(e2)=0; SF_F must not.

    By hand under the SF_F deletion rule (Section 3.5), z=1: row 0 bucket 0 holds
    e1 and e2, its max drops 2 -> 1 and A1[0]=1 is not above it, so it stays 1;
    row 1 bucket 0 holds only e1, its max drops 1 -> 0 and A2[0]=1 > 0 becomes 0.
    With z=2 and e1, e2 in different slots of row 0's bucket the max stays 1.
    Either way the Slim ends A1=[1,0], A2=[0,1]: q(e1)=0, q(e2)=1."""
    ex = _example()
    d, w = ex["d"], ex["w"]
    h = np.array([ex["e1_h"], ex["e2_h"]], dtype=np.uint32)
    f = np.array(slots, dtype=np.uint32)
    sk = oracle.Sketch(d, w, z)
    run = sk.seq_idx if mode == "seq" else (lambda *a, **k: sk.batch_idx(*a, b=1, **k))
    assert run(h, f) == 0
    np.testing.assert_array_equal(sk.slim(), np.array(ex["after_inserts_slim"]))
    assert run(h[:1], f[:1], ops=np.array([1], np.uint8), checked=True) == 0
    np.testing.assert_array_equal(sk.slim(), np.array([[1, 0], [0, 1]]))
    q = sk.query_idx(h)
    assert q[0] == 0
    assert q[1] == 1 and q[1] != ex["naive_delete_query_e2"]


# ---------------------------------------------------------------- P4: d = 1

@pytest.mark.parametrize("mode,b", [("seq", 0), ("batch", 1), ("batch", 5), ("batch", 200),
                                    ("batch", 10**9)])
@pytest.mark.parametrize("z", [1, 2, 4])
def test_d1_closed_form(mode, b, z):
    """With one row the minimum-raising insert makes A follow the bucket's largest Fat
    counter, and the deletion rule clamps it back (Appendix I holds with equality):
    A[0][j] = min(65535, max_k B[0][j][k]) for any turnstile stream and any schedule.
    With z = 1 the Slim row is the Fat row itself (a CM row)."""
    rng = np.random.default_rng(100 + z)
    keys, ops, _ = random_turnstile(rng, 3000, 80, 0.35)
    sk = oracle.Sketch(1, 16, z)
    assert (sk.seq(keys, ops, True) if mode == "seq" else sk.batch(keys, ops, b, True)) == 0
    h, f = sk_indices(keys, 1, 16, z)
    fat = histogram_fat(h, f, ops, 1, 16, z)
    np.testing.assert_array_equal(sk.slim(), np.minimum(fat.max(axis=2), SLIM_MAX))


# ---------------------------------------------------------------- P5: collision-free Fat

def _collision_free_keys(rng, n, d, w, z):
    """Keys such that no two share a Fat column (h, f) in any row (scikit-learn hash)."""
    taken = [set() for _ in range(d)]
    out = []
    while len(out) < n:
        k = np.uint32(rng.integers(0, 2**32))
        h, f = sk_indices(np.array([k]), d, w, z)
        cols = [int(h[0, i]) * z + int(f[0, i]) for i in range(d)]
        if any(c in taken[i] for i, c in enumerate(cols)):
            continue
        for i, c in enumerate(cols):
            taken[i].add(c)
        out.append(k)
    return np.array(out, dtype=np.uint32)


@pytest.mark.parametrize("mode,b", [("seq", 0), ("batch", 1), ("batch", 13), ("batch", 10**9)])
def test_collision_free_fat_theorem1(mode, b):
    """Theorem 1 (Section 3.5, correct-rate analysis) made exact: when the Fat has no
    collisions each Slim counter equals the largest net frequency among the keys that
    map to it (capped at 65535).  Lower bound from Appendix II, upper from Appendix I."""
    d, w, z = 3, 32, 8
    rng = np.random.default_rng(5)
    uni = _collision_free_keys(rng, 60, d, w, z)
    idx = rng.zipf(1.3, 6000) % uni.size
    keys = uni[idx]
    live = {}
    ops = np.zeros(keys.size, np.uint8)
    for t in range(keys.size):           # turn ~25% of positions into deletes of live keys
        if live and rng.random() < 0.25:
            k = list(live)[int(rng.integers(len(live)))]
            keys[t] = k
            ops[t] = 1
            live[k] -= 1
            if not live[k]:
                del live[k]
        else:
            live[int(keys[t])] = live.get(int(keys[t]), 0) + 1
    sk = oracle.Sketch(d, w, z)
    assert (sk.seq(keys, ops, True) if mode == "seq" else sk.batch(keys, ops, b, True)) == 0
    fq = exact_counts(keys, ops, uni)
    h, _ = sk_indices(uni, d, w, z)
    expect = np.zeros((d, w), dtype=np.int64)
    for e in range(uni.size):
        for i in range(d):
            expect[i, h[e, i]] = max(expect[i, h[e, i]], fq[e])
    np.testing.assert_array_equal(sk.slim(), np.minimum(expect, SLIM_MAX))
    q_expect = np.min(np.stack([expect[i, h[:, i]] for i in range(d)]), axis=0)
    np.testing.assert_array_equal(sk.query(uni), np.minimum(q_expect, SLIM_MAX))


# ---------------------------------------------------------------- P6: invariants

@pytest.mark.parametrize("b", [1, 3, 50])
def test_invariants_after_every_batch(b):
    """Appendix I: A_i[j] <= max_k B_i[j][k].  Appendix II: no under-estimation,
    q(e) >= min(f(e), 65535).  Also sum_j A_i[j] <= sum_j max_k B_i[j][k] <= net weight."""
    rng = np.random.default_rng(b)
    keys, ops, uni = random_turnstile(rng, 1500, 120, 0.3)
    d, w, z = 3, 16, 4
    sk = oracle.Sketch(d, w, z)
    net = 0
    for lo in range(0, keys.size, b):
        k, o = keys[lo:lo + b], ops[lo:lo + b]
        assert sk.batch(k, o, b, True) == 0
        net += int((o == 0).sum() - (o == 1).sum())
        A, B = sk.slim().astype(np.int64), sk.fat().astype(np.int64)
        assert (A <= B.max(axis=2)).all()
        f = exact_counts(keys[:lo + b], ops[:lo + b], uni)
        assert (sk.query(uni) >= np.minimum(f, SLIM_MAX)).all()
        assert (A.sum(axis=1) <= B.max(axis=2).sum(axis=1)).all()
        assert (B.max(axis=2).sum(axis=1) <= net).all()


def test_alpha_at_most_one_insert_only():
    """Section 3.5 error bound: at most one Slim counter per array is incremented per
    insertion, so alpha = sum(A) / (d * N) <= 1 for insert-only sequential streams."""
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 500, 20000).astype(np.uint32)
    sk = oracle.Sketch(4, 64, 4)
    sk.seq(keys)
    alpha = sk.slim().astype(np.int64).sum() / (4 * keys.size)
    assert 0 < alpha <= 1


# ---------------------------------------------------------------- P7, P8: cross-checks

def test_batch_of_one_is_sequential():
    """The batch schedule with one op per batch is the sequential rule (two code paths)."""
    rng = np.random.default_rng(21)
    for trial in range(200):
        d = int(rng.integers(1, 6))
        w, z = int(rng.choice([2, 4, 8, 5])), int(rng.choice([1, 2, 3, 4]))
        keys, ops, _ = random_turnstile(rng, int(rng.integers(1, 400)), 20, 0.3)
        a, b = oracle.Sketch(d, w, z), oracle.Sketch(d, w, z)
        assert a.seq(keys, ops, True) == 0 and b.batch(keys, ops, 1, True) == 0
        np.testing.assert_array_equal(a.slim(), b.slim())
        np.testing.assert_array_equal(a.fat(), b.fat())


def test_c_oracle_matches_python_transcription():
    """The C oracle and the pure-Python transcription (different language, different
    hash code) agree on 10^4 tiny random turnstile streams, sequential mode, plus the
    batch schedule at several b, with brute-force counts as the no-under-estimate floor."""
    rng = np.random.default_rng(2024)
    for trial in range(10_000):
        d = int(rng.integers(1, 5))
        w, z = int(rng.choice([2, 4, 8])), int(rng.choice([1, 2, 4]))
        n = int(rng.integers(1, 200 if trial % 10 == 0 else 40))
        keys, ops, uni = random_turnstile(rng, n, int(rng.integers(1, 16)), 0.3)
        c = oracle.Sketch(d, w, z)
        assert c.seq(keys, ops, True) == 0
        p = sfpy.SF(d, w, z)
        p.seq(zip(keys.tolist(), ops.tolist()))
        assert c.slim().tolist() == p.A and c.fat().tolist() == p.B
        assert (c.query(uni) >= exact_counts(keys, ops, uni)).all()
        if trial % 20 == 0:
            for b in (2, 5, 64):
                c = oracle.Sketch(d, w, z)
                assert c.batch(keys, ops, b, True) == 0
                p = sfpy.SF(d, w, z)
                p.batch(zip(keys.tolist(), ops.tolist()), b)
                assert c.slim().tolist() == p.A and c.fat().tolist() == p.B


def test_flow_keys_match_python_transcription():
    """13-byte keys hash as their raw bytes in both transcriptions."""
    rng = np.random.default_rng(9)
    keys, ops, uni = random_turnstile(rng, 300, 30, 0.3, key_bytes=13)
    c = oracle.Sketch(4, 8, 4, key_bytes=13)
    assert c.seq(keys, ops, True) == 0
    p = sfpy.SF(4, 8, 4)
    p.seq(zip([bytes(k) for k in keys], ops.tolist()))
    assert c.slim().tolist() == p.A and c.fat().tolist() == p.B


# ---------------------------------------------------------------- single key, saturation

@pytest.mark.parametrize("c", [1, 2, 9, 100])
def test_single_key_water_level(c):
    """c inserts of one key in one batch reach the same Slim state as c sequential
    inserts, from a non-trivial start state (prefix of other keys)."""
    rng = np.random.default_rng(c)
    pre = rng.integers(0, 50, 400).astype(np.uint32)
    key = np.full(c, 7, dtype=np.uint32)
    a, b = oracle.Sketch(3, 8, 2), oracle.Sketch(3, 8, 2)
    a.seq(pre)
    b.seq(pre)
    a.seq(key)
    b.batch(key, None, c)
    np.testing.assert_array_equal(a.slim(), b.slim())


@pytest.mark.parametrize("mode", ["seq", "batch"])
def test_slim_saturates_at_65535(mode):
    """uint16 Slim: a key with 70000 occurrences reads 65535 ("at least 65535"); its
    Fat counters hold the exact 70000; deleting 10000 clamps its cells to 60000."""
    keys = np.full(70000, 12345, dtype=np.uint32)
    sk = oracle.Sketch(2, 8, 2)
    run = (lambda k, o=None: sk.seq(k, o, True)) if mode == "seq" else \
        (lambda k, o=None: sk.batch(k, o, 4096, True))
    assert run(keys) == 0
    assert sk.query(keys[:1])[0] == SLIM_MAX
    h, f = sk_indices(keys[:1], 2, 8, 2)
    assert all(sk.fat()[i, h[0, i], f[0, i]] == 70000 for i in range(2))
    assert run(keys[:10000], np.ones(10000, np.uint8)) == 0
    assert sk.query(keys[:1])[0] == 60000


def test_checked_mode_rejects_underflow():
    """Deleting a key that was never inserted violates the strict-turnstile
    precondition of Appendix II; the checked mode reports it."""
    for run in ("seq", "batch"):
        sk = oracle.Sketch(2, 8, 2)
        sk.seq(np.array([1, 2], np.uint32))
        k = np.array([99], np.uint32)
        o = np.array([1], np.uint8)
        rc = sk.seq(k, o, True) if run == "seq" else sk.batch(k, o, 1, True)
        assert rc == oracle.EUNDERFLOW


# ---------------------------------------------------------------- P10, full-size C1

def _bounds(sk_fat, h, f_true):
    U = np.min(np.stack([sk_fat[i][h[:, i]].max(axis=1) for i in range(h.shape[1])]), axis=0)
    return U.astype(np.int64), np.minimum(f_true, SLIM_MAX)


def test_intermode_bound_small_config():
    """Both modes answer inside [min(f,65535), U(e)] with U(e) = min_i max_k B_i[h_i][k]
    (Appendices I and II) and share the same Fat, so |q_batch - q_seq| <= U - f' for
    every key.  Run on the small configuration (1M Zipf(1.0) inserts, d=4, w=16384,
    z=4), which also pins the Fat against the scikit-learn histogram at full size."""
    import sfgen
    wl = sfgen.config_small()
    seq = oracle.Sketch(wl.d, wl.w, wl.z)
    seq.seq(wl.keys)
    bat = oracle.Sketch(wl.d, wl.w, wl.z)
    bat.batch(wl.keys, None, 65536)
    fat = seq.fat()
    np.testing.assert_array_equal(fat, bat.fat())
    h, f = sk_indices(wl.keys, wl.d, wl.w, wl.z)
    np.testing.assert_array_equal(fat, histogram_fat(h, f, None, wl.d, wl.w, wl.z))
    f_true = exact_counts(wl.keys, None, wl.queries)
    hq, _ = sk_indices(wl.queries, wl.d, wl.w, wl.z)
    U, fp = _bounds(fat, hq, f_true)
    qs, qb = seq.query(wl.queries).astype(np.int64), bat.query(wl.queries).astype(np.int64)
    for q in (qs, qb):
        assert (q >= fp).all() and (q <= U).all()
    assert (np.abs(qb - qs) <= U - fp).all()


def test_error_bound_markov_small_config():
    """Section 3.5 over-estimation bound, read with e = exp(1): the fraction of keys
    with f_hat >= f + e*alpha*N/w is at most e^-d (d=4: 1.83%), alpha = sum A/(d N).
    Statistical, so allow one percentage point of slack."""
    import sfgen
    wl = sfgen.config_small()
    sk = oracle.Sketch(wl.d, wl.w, wl.z)
    sk.seq(wl.keys)
    alpha = sk.slim().astype(np.int64).sum() / (wl.d * wl.n_ops)
    f_true = exact_counts(wl.keys, None, wl.queries)
    q = sk.query(wl.queries).astype(np.int64)
    present = f_true > 0
    err = q[present] - f_true[present]
    frac = np.mean(err >= math.e * alpha * wl.n_ops / wl.w)
    assert frac <= math.exp(-wl.d) + 0.01
