"""The C ABI library loads and exports what include/sf.h declares; host-side
validation and budget checks run before any device call (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1701_04148_amd as sf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 14
    L = ctypes.CDLL(sf.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sf.SIGNATURES)


def test_strerror_texts():
    assert sf.sf_strerror(0) == "ok"
    for code in (-1, -2, -3, -4, -5):
        assert sf.sf_strerror(code) and sf.sf_strerror(code) != "unknown status"
    assert sf.sf_strerror(-99) == "unknown status"


@pytest.mark.parametrize("bad", [dict(d=0), dict(d=17), dict(w=0), dict(z=0), dict(key_bytes=8),
                                 dict(batch_ops=0), dict(w=1 << 31, z=4)])
def test_invalid_config_rejected_before_device(bad):
    cfg = dict(d=4, w=1024, z=4, key_bytes=4, seed_base=1, batch_ops=1024)
    cfg.update(bad)
    c = sf.make_config(**cfg)
    assert sf.sf_footprint(c) == 0
    h = ctypes.c_void_p()
    rc = sf.lib().sf_create(ctypes.byref(c), 0, None, ctypes.byref(h))
    assert rc == sf.SF_EINVAL and not h.value
    assert sf.sf_last_error()


def test_footprint_and_budget():
    c = sf.make_config(4, 1 << 20, 4, 4, 1, 1 << 21)
    fp = sf.sf_footprint(c)
    cells = 4 << 20
    b = 1 << 21
    merge = b * 4 + b * 4 + b * 4          # partitioned keys, entry keys, entry counts
    # cell records (z Fat counters + Slim), export staging (dense Fat), dense uint16 Slim
    # copy for queries, snapshots, merge buffers
    hist = (b // 8192 + 1) * 2048 * 4      # per-partition-group bucket histograms (2 x 1024 buckets)
    chunks = (b // 2048 + 2 * 1024 + 1) * 20   # every merge chunk: key range, whole buckets
    meta = 4 * (2 * 1024 + 1) * 4 + 3 * 256     # per-bucket totals, starts, sizes, chunk prefix; counters
    need = cells * 5 * 4 + cells * 4 * 4 + cells * 2 + 4 * b * 6 + merge + hist + chunks
    # owner-computes S1..S5 (this shape qualifies: 1024 ranges of 1024 cells per row):
    # pairs of two batches, their positions, per-pair snapshots, T per entry, per-tile
    # column counts (b / 4096 tiles); column starts of three batches
    ncol = 2 * 4 * 1024
    owner = 2 * 4 * b * 8 + 4 * b * 4 + 4 * b * 8 + b * 2 + (b // 4096) * ncol * 4
    pair_meta = 3 * (2 * 16384 + 3) * 4       # column totals and starts, entry counts (3 batches)
    need += owner
    assert fp >= need
    assert fp < need + meta + pair_meta + (8 << 10)          # plus 256-B rounding
    h = ctypes.c_void_p()
    rc = sf.lib().sf_create(ctypes.byref(c), fp - 1, None, ctypes.byref(h))
    assert rc == sf.SF_ENOMEM and not h.value
    assert "budget" in sf.sf_last_error()


def test_dead_handles_rejected():
    for fn in ("sf_destroy", "sf_sync", "sf_reset", "sf_merge_path", "sf_owner_range", "sf_group_merge_path",
               "sf_group_destroy", "sf_pool_destroy"):
        assert getattr(sf.lib(), fn)(None) == sf.SF_ESTATE, fn
    assert sf.lib().sf_set_streams(None, 0) == sf.SF_ESTATE
    assert sf.lib().sf_set_owner_range(None, 0) == sf.SF_ESTATE
    assert sf.lib().sf_group_set_owner_ratio(None, 1.0) == sf.SF_ESTATE
    assert sf.lib().sf_group_set_merge(None, 1) == sf.SF_ESTATE
    assert sf.lib().sf_insert(None, None, 0) == sf.SF_ESTATE
    assert sf.lib().sf_query(ctypes.c_void_p(12345), None, 0, None) == sf.SF_ESTATE
