#!/usr/bin/env python3
"""SF-sketch hot-path benchmark on one MI355X.

One step = the whole hot path over one batch of synthetic input, with keys
already resident in HBM: re-zero the sketch, apply the op stream (inserts and
deletes through the deterministic batch schedule), export the Slim (what the
monitor ships to the collector), and answer the point queries.

Headline workload: one SF-sketch, d=4, Fat 4 x 2^22 uint32 (w=2^20 buckets
of z=4), Slim 4 x 2^20 uint16; 32M uint32 ops, Zipf(s=1.0) over 1M distinct
keys, 10% deletions of live occurrences; queries = the 1M keys + 1M absent.
Further legs, each timed the same way and checked against the CPU oracle at
full size: the same workload at Zipf 0.6 and 1.4, the 1M-insert sketch
(d=4, w=2^14), the 128M-packet flow sketch (d=8, w=2^21, 13-byte keys), 1024
sketches in one group, and the serving loop.

Prints ONE JSON line (rank 0): throughput in M items/s (ops + queries), the
dominant kernel's roofline object, the CPU oracle timed on the host (batch
and sequential updates on one core, queries on one core and on all cores),
and the batch schedule's accuracy against sequential SF_F.  Progress goes to
stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Minsert+query items/s per GPU (1 vs 1024 sketches); p50/p99 served latency"
HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")

from paper_1701_04148_amd.tune import batch_for_width  # noqa: E402  (the b rule, shared with the tests)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    """Digest of the kernel sources; a stored counter reading is valid only for it."""
    h = hashlib.sha256()
    for rel in ("paper_1701_04148_amd/csrc/sf_lib.hip", "paper_1701_04148_amd/csrc/sf_device.hpp",
                "paper_1701_04148_amd/csrc/sf_kernels.hpp", "paper_1701_04148_amd/csrc/sf_host.hpp",
                "paper_1701_04148_amd/csrc/sf_owner.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kind: str, d: int, u: dict, kb: int = 4) -> int:
    """Bytes one kernel kind's step must move over the timed steps, each access counted
    at its element size.  u holds the units: ins / dels / ops (op counts), q (queries),
    ie / de (merged insert / delete entries; equal to ins / dels when merging per tile),
    cells, mixed (1 B op code per op); kb = key bytes.  The owner step (k_own_step, its
    kinds own_step and own_final) does S1..S5 of every entry: per row an insert entry
    reads and writes its Fat counter and reads and may write its Slim counter (12 B), a
    delete entry reads and writes its Fat counter, reads the rest of its bucket (12 B)
    and reads and may write its Slim counter (24 B)."""
    ob = u["ops"] if u["mixed"] else 0
    own = u["ie"] * d * 12 + u["de"] * d * 24
    return {
        "partition": (u["ins"] + u["dels"]) * (3 * kb) + 2 * ob,  # keys read twice, partitioned copy written
        "merge": (u["ins"] + u["dels"]) * kb + (u["ie"] + u["de"]) * (kb + 4),  # partitioned keys in, entries out
        "pairs": (u["ie"] + u["de"]) * (2 * (kb + 4) + d * 8) + u["ie"] * d * 4,  # entries read twice, pairs out
        "own_step": own, "own_final": own,                   # (split by launches below)
        "level": u["ie"] * (d * (4 + 8) + 2),                # positions, pair snapshots, T out
        "snapshot": u["ie"] * (kb + d * (4 + 4 + 4 + 2)),    # key, Slim cell, Fat counter, snapshot out
        "fat_add": u["ie"] * (kb + 4 + d * 8),               # key + count, Fat read-modify-write
        "raise": u["ie"] * (kb + d * (4 + 4 + 2)),           # key, Fat counter, snapshot in
        "fat_sub": u["de"] * (kb + 4 + d * 8),
        "clamp": u["de"] * (kb + d * (16 + 4)),              # key, 16-B bucket, Slim cell
        "query": u["q"] * (kb + d * 4 + 4),                  # key, d Slim cells, answer
        "export": u["cells"] * 6,                            # 4-B working cell in, 2-B cell out
    }.get(kind, 0)


def random_accesses(kind: str, d: int, u: dict) -> int:
    """Random (uncoalesced) accesses of a kernel kind over the timed steps: one per cell
    record touched (a record holds the cell's Fat bucket and Slim word), one per atomic.
    The owner path has none on the records (its ranges are staged in LDS)."""
    return {"snapshot": d * u["ie"], "fat_add": d * u["ie"], "raise": 2 * d * u["ie"],
            "fat_sub": d * u["de"], "clamp": 2 * d * u["de"], "query": d * u["q"],
            "level": d * u["ie"]}.get(kind, 0)


def step_algorithmic_bytes(d: int, n_ins: int, n_del: int, n_q: int, kb: int = 4) -> int:
    """The method's own bytes per op, whatever the implementation: an insert touches the
    key, d Fat counters (read-modify-write) and d Slim cells; a delete the key, d Fat
    buckets and d Slim cells; a query the key and d Slim cells (uint16).  With 13-byte
    keys and d = 8: 93 B per insert, 29 B per query."""
    return n_ins * (kb + d * 8 + d * 2) + n_del * (kb + d * (8 + 12) + d * 2) + n_q * (kb + 2 * d)


def stored_traffic(kernel_kind: str, workload: str):
    """HBM bytes per launch from the committed PMC summary, if taken on these sources and
    this workload."""
    path = os.path.join(PROFILE_DIR, "pmc_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    k = rec.get("workloads", {}).get(workload, {}).get("kernels", {}).get(kernel_kind)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


KIND_OF_KERNEL = {"k_own_step": "own_step", "k_level": "level", "k_pair_count": "pair_count",
                  "k_pair_colscan": "pair_colscan", "k_pair_start": "pair_start", "k_pair_scatter": "pair_scatter",
                  "k_snapshot": "snapshot", "k_raise": "raise", "k_clamp": "clamp",
                  "k_query": "query", "k_query_rows": "query", "k_query_min": "query", "k_pack16": "export", "k_merge": "merge",
                  "k_entries_snapshot": "snapshot", "k_entries_snapshot_rows": "snapshot",
                  "k_entries_raise": "raise", "k_entries_clamp": "clamp",
                  "k_part_count": "part_count", "k_part_colscan": "part_colscan", "k_part_colscan_tall": "part_colscan", "k_part_start": "part_start",
                  "k_unpack_fat": "fat_export",
                  "k_part_scatter": "part_scatter"}


def _kernel_base(name: str) -> str:
    """Bare kernel name: no return type, namespace, template or argument list."""
    base = name.replace("(anonymous namespace)::", "").replace("void ", "").strip()
    return base.split("(")[0].split("<")[0].strip().split("::")[-1]


def summarize_pmc(fetch_csv: str, write_csv: str, workload: str, copy_bytes: int) -> dict:
    """Per-kernel HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), scaled so the plain copy kernel reads and writes
    exactly copy_bytes.  k_fat_update dispatches alternate add / subtract within a
    batch (add follows the snapshot, subtract follows the raise)."""
    import csv
    from collections import defaultdict

    def per_kind(path, counter):
        rows = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                rows.append((int(r.get("Dispatch_Id", 0)), _kernel_base(r["Kernel_Name"]),
                             float(r["Counter_Value"])))
        rows.sort()
        vals, prev = defaultdict(list), None
        for _, base, v in rows:
            if base in ("k_fat_update", "k_entries_fat"):
                kind = "fat_sub" if prev in ("k_raise", "k_entries_raise") else "fat_add"
            else:
                kind = KIND_OF_KERNEL.get(base, base)
            vals[kind].append(v)
            prev = base
        return {k: sum(v) / len(v) for k, v in vals.items()}

    fetch, write = per_kind(fetch_csv, "FETCH_SIZE"), per_kind(write_csv, "WRITE_SIZE")
    f_scale = (copy_bytes / 1024.0) / fetch["k_copy"]
    w_scale = (copy_bytes / 1024.0) / write["k_copy"]
    kernels = {}
    for kind in fetch:
        if kind == "k_copy" or kind not in write:
            continue
        rd, wr = fetch[kind] * f_scale * 1024, write[kind] * w_scale * 1024
        kernels[kind] = {"fetch_kib_raw": round(fetch[kind], 1), "write_kib_raw": round(write[kind], 1),
                         "hbm_bytes_per_launch": int(rd + wr)}
    return {"workload": workload, "source_digest": source_digest(),
            "copy_calibration": {"bytes": copy_bytes, "fetch_scale": round(f_scale, 4),
                                 "write_scale": round(w_scale, 4)},
            "kernels": kernels}


def format_pmc(rec: dict) -> str:
    """Text table of one workload's PMC record (raw KiB per dispatch, calibrated bytes)."""
    lines = [f"# workload {rec['workload']}; kernel sources digest {rec['source_digest']}",
             f"# calibration: a plain {rec['copy_calibration']['bytes']} B copy kernel: FETCH_SIZE x "
             f"{rec['copy_calibration']['fetch_scale']}, WRITE_SIZE x {rec['copy_calibration']['write_scale']}",
             f"{'kernel':16s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s} {'bytes/launch(calibrated)':>26s}"]
    for k, v in sorted(rec["kernels"].items(), key=lambda kv: -kv[1]["hbm_bytes_per_launch"]):
        lines.append(f"{k:16s} {v['fetch_kib_raw']:12.1f} {v['write_kib_raw']:12.1f} {v['hbm_bytes_per_launch']:26,d}")
    return "\n".join(lines)


def store_pmc(rec: dict, path: str = "") -> dict:
    """Adds one workload's PMC record to the PMC summary file (profiles/pmc_traffic.json by
    default; records taken on other kernel sources are dropped)."""
    path = path or os.path.join(PROFILE_DIR, "pmc_traffic.json")
    try:
        with open(path) as fh:
            allrec = json.load(fh)
    except (OSError, ValueError):
        allrec = {}
    if allrec.get("source_digest") != rec["source_digest"]:
        allrec = {"source_digest": rec["source_digest"], "workloads": {}}
    allrec.setdefault("workloads", {})[rec["workload"]] = {
        "copy_calibration": rec["copy_calibration"], "kernels": rec["kernels"]}
    with open(path, "w") as fh:
        json.dump(allrec, fh, indent=1)
    return allrec


def summarize_stats(stats_csv: str) -> str:
    """Text table of a rocprofv3 --stats kernel_stats.csv (per-kernel calls and durations)."""
    import csv
    rows = []
    with open(stats_csv) as fh:
        for r in csv.DictReader(fh):
            name = r["Name"].replace("(anonymous namespace)::", "").replace("void ", "")
            name = name.replace("sfk::", "").split("(")[0]
            rows.append((name[:44], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                         float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                         float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    lines = [f"{'kernel':44s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}"]
    for n, c, t, a, lo, hi, pct in rows:
        lines.append(f"{n:44s} {c:6d} {t:9.3f} {a:8.1f} {lo:8.1f} {hi:8.1f} {pct:6.2f}")
    return "\n".join(lines)


def summarize_trace(trace_csv: str) -> str:
    """Per-kind kernel durations from a rocprofv3 kernel_trace.csv, with the Fat kernel's
    insert (S2) and delete (S4) dispatches told apart by the kernel before them -- the
    kinds and units bench.py's event timing reports."""
    import csv
    from collections import defaultdict
    rows = []
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _kernel_base(r["Kernel_Name"])))
    rows.sort()
    dur, prev = defaultdict(list), None
    for t0, t1, base in rows:
        if base in ("k_fat_update", "k_entries_fat"):
            kind = "fat_sub" if prev in ("k_raise", "k_entries_raise") else "fat_add"
        else:
            kind = KIND_OF_KERNEL.get(base, base)
        dur[kind].append((t1 - t0) / 1e3)
        prev = base
    lines = [f"{'kind':16s} {'dispatches':>10s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s}"]
    for kind, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{kind:16s} {len(v):10d} {sum(v) / len(v):8.1f} {min(v):8.1f} {max(v):8.1f}")
    return "\n".join(lines)


def workload_tag(leg: str, b: int, scale: int = 1) -> str:
    """Name of a timed workload (sketch shape, stream, schedule) for stored counters."""
    return f"{leg}_b{b}_scale{scale}"


def cpu_info() -> dict:
    """The host the CPU oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        aff = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "affinity_cpus": aff,
            "threads_for_all_cores": min(16, aff)}


def micro_ceilings(torch, sizes_mib=(1, 16, 64, 256, 4096), n=1 << 26):
    """Measured random-access ceilings (G accesses/s) at several footprints."""
    from paper_1701_04148_amd import micro
    out = {}
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    for mib in sizes_mib:
        elems = (mib << 20) // 4
        t = torch.zeros(elems, dtype=torch.int32, device="cuda")
        res = {}
        for name, fn in (("gather_u32", lambda s: micro.gather_u32(t, n, s, sink)),
                         ("atomic_add_u32", lambda s: micro.atomic_add_u32(t, n, s)),
                         ("gather_16b", lambda s: micro.gather_16b(t, n, s, sink)),
                         ("pair_same_line", lambda s: micro.gather_pair(t, n, s, True, sink)),
                         ("pair_two_lines", lambda s: micro.gather_pair(t, n, s, False, sink)),
                         ("scatter_u64", lambda s: micro.scatter_u64(t.view(torch.int64), n, s))):
            fn(1)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for s in range(3):
                fn(100 + s)
            e1.record()
            torch.cuda.synchronize()
            res[name] = round(3 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9, 2)
        out[f"{mib}MiB"] = res
        del t
        torch.cuda.empty_cache()
    return out


def lone_compare(args, torch, np, sf, cfgs, keys, ops, qk, out, m, group_answers):
    """The plain path: one Sketch per stream, its own launches (the atomic S1..S5 path,
    one sketch and one batch per launch); its answers must equal the group's."""
    lone = [sf.Sketch(c.d, c.w, c.z, batch_ops=c.batch_ops) for c in cfgs]
    for s_ in lone:
        # the group's kernels, one sketch and one batch per launch (the owner-computes path
        # would also need its pair buffers per sketch)
        s_.set_tile(args.tile)
        s_.set_merge(2 if args.merge != "tile" else 0)
    seg, qseg = m.seg.astype(np.int64), m.qseg.astype(np.int64)

    def lone_step():
        for i, s_ in enumerate(lone):
            s_.reset()
            s_.update(keys[seg[i]:seg[i + 1]], ops[seg[i]:seg[i + 1]])
            s_.query(qk[qseg[i]:qseg[i + 1]], out[qseg[i]:qseg[i + 1]])

    lone_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lone_step()
    torch.cuda.synchronize()
    el1 = time.perf_counter() - t0
    lone_value = (int(m.keys.size) + int(m.queries.size)) / el1 / 1e6
    same = bool(np.array_equal(out.cpu().numpy().view(np.uint32), group_answers))
    log(f"[bench] one sketch per launch: {el1 * 1e3:.2f} ms/step, {lone_value:.1f} M items/s; "
        f"answers identical to the group: {same}")
    for s_ in lone:
        s_.close()
    if not same:
        raise SystemExit("group answers differ from the one-sketch-per-launch path")
    return lone_value, el1


def run_multi(args, torch, np, sf, sfgen):
    """1024 sketches in one group (graph-captured rounds) vs one sketch per launch."""
    t_gen = time.time()
    m = sfgen.config_multi(seed=0, length_scale=1.0 / args.scale,
                           workers=args.gen_workers or min(16, os.cpu_count() or 1))
    n_ops, n_q = int(m.keys.size), int(m.queries.size)
    log(f"[bench] workload {m.name}: {m.n} sketches, {n_ops} ops ({int(m.ops.sum())} deletes), "
        f"{n_q} queries, generated in {time.time() - t_gen:.1f}s")
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(m.keys.view(np.int32)).to(dev)
    ops = torch.from_numpy(m.ops).to(dev)
    qk = torch.from_numpy(m.queries.view(np.int32)).to(dev)
    out = torch.empty(n_q, dtype=torch.int32, device=dev)
    batch_of_w = {int(w): batch_for_width(int(w)) for w in np.unique(m.w)}
    tuned = None
    fixed = None
    if args.multi_shape_in:
        # a shape an earlier autotuned run wrote (profiling runs replay it without tuning)
        with open(args.multi_shape_in) as f:
            fixed = json.load(f)
        batch_of_w.update({int(w): int(b) for w, b in fixed["batch_of_w"].items()})
        log(f"[bench] group shape from {args.multi_shape_in}: {fixed}")
    elif not args.no_autotune:
        # one tuning run per sketch width on that class's longest stream (at most 2M ops)
        from paper_1701_04148_amd.tune import tune_batch
        t_tune = time.time()
        lens = np.diff(m.seg.astype(np.int64))
        tuned = {}
        for w in sorted(batch_of_w):
            i = int(np.argmax(np.where(m.w == w, lens, -1)))
            k_i, o_i, q_i = m.part(i)
            n = min(k_i.shape[0], 1 << 21)
            # b is the same whichever path runs the group (the answers do not depend on it);
            # the atomic path's time of a lone sketch stands in for the group's per-width cost
            r = tune_batch(m.d, w, m.z, k_i[:n], o_i[:n], q_i, modes=(2,))
            batch_of_w[w] = r.b
            tuned[str(w)] = {"b": r.b, "rule_b": batch_for_width(w), "ref_b": r.ref_b,
                             "ref_are": round(r.ref_are, 5), "bound": round(r.bound, 5),
                             "candidates": [[b, round(a, 5), round(ms, 2), ok] for b, a, ms, ok, _, _ in r.table]}
        log(f"[bench] autotuned batch per width in {time.time() - t_tune:.1f}s: "
            f"{ {w: v['b'] for w, v in tuned.items()} } (rule min(16 w, 2^23): "
            f"{ {w: v['rule_b'] for w, v in tuned.items()} })")
    cfgs = [sf.make_config(m.d, int(m.w[i]), m.z, 4, 1, batch_of_w[int(m.w[i])]) for i in range(m.n)]
    group_mode = {"tile": 0, "batch": 1, "owner": 1, "atomic": 2}[args.merge]
    round_ops = args.group_round_ops
    owner_ratio = args.group_owner_ratio
    shape = None
    if fixed is not None:
        group_mode, round_ops = int(fixed["mode"]), int(fixed["round_ops"])
        owner_ratio = float(fixed.get("owner_ratio", 0.0))
    elif not args.no_autotune and args.merge == "batch" and not round_ops:
        # the group's merge path and launch-round size, timed on its own streams
        from paper_1701_04148_amd.tune import tune_group
        t_tune = time.time()
        gs = tune_group(cfgs, keys, ops, m.seg)
        group_mode, round_ops, owner_ratio = gs.mode, gs.round_ops, gs.ratio
        shape = {"mode": gs.mode, "owner_ratio": gs.ratio, "round_ops": gs.round_ops,
                 "candidates": [[md, ra, r, round(ms, 2), sub] for md, ra, r, ms, sub in gs.table]}
        log(f"[bench] autotuned group shape in {time.time() - t_tune:.1f}s: path {gs.mode}, owner ratio "
            f"{gs.ratio}, round_ops {gs.round_ops} (candidates [path, owner ratio, round_ops, ms, launch "
            f"rounds]: {shape['candidates']})")
    if args.multi_shape_out:
        with open(args.multi_shape_out, "w") as f:
            json.dump({"batch_of_w": {str(w): b for w, b in batch_of_w.items()}, "mode": group_mode,
                       "owner_ratio": owner_ratio, "round_ops": round_ops}, f)
    G = sf.SketchGroup(cfgs, round_ops=round_ops)
    G.set_tile(args.tile)
    G.set_merge(group_mode)
    if G.merge_path() == 1:
        G.set_owner_ratio(owner_ratio)
    path = G.merge_path()
    log(f"[bench] group merge path {path} (0 per tile, 1 owner-computes, 2 atomics)")

    def step():
        G.reset()
        G.update(keys, ops, m.seg)
        G.query(qk, m.qseg, out)

    for _ in range(args.warmup):
        step()
    G.sync()
    torch.cuda.synchronize()
    ie0, de0 = G.merge_stats()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    G.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ie1, de1 = G.merge_stats()
    ms_step = el * 1e3 / args.steps
    value = (n_ops + n_q) * args.steps / el / 1e6
    sub, tiles = G.rounds()
    entries = ((ie1 - ie0) // args.steps, (de1 - de0) // args.steps)
    log(f"[bench] group: {ms_step:.2f} ms/step, {value:.1f} M items/s ({sub} launch rounds, {tiles} tiles, "
        f"merged entries per step: {entries[0]} inserts, {entries[1]} deletes)")
    # per-kernel times from one profiled (eager) pass
    G.profile(True)
    G.profile_read(reset=True)
    step()
    prof = G.profile_read(reset=True)
    G.profile(False)
    kernels = {k: dict(ms=round(v[0], 3), launches=v[1]) for k, v in prof.items() if v[1]}
    rows = []
    for i in range(0, m.n, max(1, m.n // 8)):       # sanity: Fat row sums = net weight
        k_i, o_i, _ = m.part(i)
        net = int((o_i == 0).sum()) - int((o_i == 1).sum())
        fat = G.export_fat(i)
        rows.append(bool((fat.reshape(m.d, -1).astype(np.int64).sum(axis=1) == net).all()))
    if not all(rows):
        raise SystemExit("group Fat row sums differ from net stream weight")
    group_answers = out.cpu().numpy().view(np.uint32).copy()
    G.close()
    del G
    torch.cuda.empty_cache()

    if args.no_lone_compare:
        lone_value, el1 = None, None
    else:
        lone_value, el1 = lone_compare(args, torch, np, sf, cfgs, keys, ops, qk, out, m, group_answers)
    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mitems/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{m.n} SF-sketches, d=4, Fat 2^14..2^20 u32 log-uniform (z=4), "
                               "stream lengths lognormal median 200K in [10K, 4M], Zipf(1.1), 5% deletes; "
                               "one graph-captured group update, then query every stream's universe",
                   "sketches": m.n, "ops": n_ops, "queries": n_q,
                   "batch_ops": ("autotuned per width" if tuned else "min(16 w, 2^23) per sketch"),
                   "tile_ops": args.tile, "merge": args.merge, "merge_path": path, "owner_ratio": owner_ratio,
                   "round_ops": round_ops,
                   "launch_rounds": sub, "scale": args.scale},
        "merged_entries_per_step": {"insert": entries[0], "delete": entries[1]},
        "autotune": tuned,
        "group_shape": shape,
        "one_sketch_per_launch": None if lone_value is None else {
            "value": round(lone_value, 2), "unit": "Mitems/s", "ms_per_step": round(el1 * 1e3, 3)},
        "group_vs_lone": None if lone_value is None else round(value / lone_value, 2),
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        import oracle
        n_s = 0
        c0 = time.perf_counter()
        items = 0
        while n_s < m.n and time.perf_counter() - c0 < 15.0:
            k_i, o_i, q_i = m.part(n_s)
            ref = oracle.Sketch(m.d, int(m.w[n_s]), m.z)
            ref.batch(k_i, o_i, cfgs[n_s].batch_ops)
            ans = ref.query(q_i)
            q0, q1 = int(m.qseg[n_s]), int(m.qseg[n_s + 1])
            if not np.array_equal(ans, group_answers[q0:q1]):
                raise SystemExit(f"sketch {n_s}: GPU answers differ from the oracle")
            items += k_i.shape[0] + q_i.shape[0]
            n_s += 1
        c_el = time.perf_counter() - c0
        result["cpu_baseline"] = {"value": round(items / c_el / 1e6, 3), "unit": "Mitems/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"first {n_s} of {m.n} sketches ({items} ops + queries), "
                                            f"{c_el:.1f}s on 1 thread; their GPU answers bit-exact"}
    return result


SERVE_SHAPES = {
    # per-stream sketch "as the 128M-packet flow configuration": d=8, Fat 8 x 2^23, Slim 8 x 2^21
    "flows": dict(d=8, w=1 << 21, z=4),
    # the many-sketch configuration's largest sketch: d=4, Fat 4 x 2^20, Slim 4 x 2^18
    "small": dict(d=4, w=1 << 18, z=4),
}


def serve_workload(args, sfgen):
    t_gen = time.time()
    w = sfgen.serving(seed=0, n_streams=4096 // args.scale, per_stream=16)
    log(f"[bench] serving workload: {len(w.requests)} requests, {w.n_streams} streams, "
        f"{sum(r.n for r in w.requests)} keys, generated in {time.time() - t_gen:.1f}s")
    return w


def run_serve(args, torch, np, sf, sfgen, shape_name, w=None):
    """4096 streams of insert/delete/query requests through the continuous-batching loop:
    the saturation rate (every request visible at once), then arrivals replayed at each
    offered load of --serve-loads (fractions of saturation) with per-kind latency, and a
    sample of streams checked against the CPU oracle (their closing Slim and every query
    answer)."""
    from paper_1701_04148_amd.serve import Server
    if w is None:
        w = serve_workload(args, sfgen)
    total_keys = sum(r.n for r in w.requests)
    shape = SERVE_SHAPES[shape_name]
    cfg = sf.make_config(shape["d"], shape["w"], shape["z"], 4, 1, batch_for_width(shape["w"]))
    budget = 64 << 30
    pool = sf.SketchPool(cfg, hbm_budget_bytes=budget)
    pool.set_merge(args.merge != "tile")
    owner_ratio = None
    if args.merge != "tile":
        try:
            pool.set_owner_ratio(args.pool_owner_ratio)
            owner_ratio = args.pool_owner_ratio
        except sf.SFError:
            pass  # slots too large for the owner path: atomic entry kernels throughout
    slots, _ = pool.capacity()
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(w.pool.view(np.int32)).to(dev)
    # a delete's keys (its pieces of the pool) joined on the device before the loop starts
    joined = {(r.stream, r.seq): torch.cat([keys[o:o + c] for o, c in r.pieces]) for r in w.requests if r.pieces}
    torch.cuda.synchronize()
    answers = torch.empty(1 << 20, dtype=torch.int32, device=dev)          # answers are discarded ...
    sink = torch.empty(shape["d"] * shape["w"], dtype=torch.int16, device=dev)  # stands for the collector
    check = sorted({0, w.n_streams // 2, w.n_streams - 1})                # ... except for these streams
    c_slim = {st: torch.zeros(shape["d"] * shape["w"], dtype=torch.int16, device=dev) for st in check}
    c_ans = {(r.stream, r.seq): torch.full((r.n,), -1, dtype=torch.int32, device=dev)
             for r in w.requests if r.stream in c_slim and r.kind == sf.SF_REQ_QUERY}
    srv = Server(pool, max_launch_keys=args.serve_launch_keys, max_in_flight=3)

    def go(reqs, realtime):
        return srv.run(reqs, key_of=lambda r: joined[(r.stream, r.seq)] if r.pieces else keys[r.off:r.off + r.n],
                       out_of=lambda r: c_ans.get((r.stream, r.seq), answers[:r.n]),
                       export_to=lambda st: c_slim.get(st, sink), realtime=realtime)

    warm = [r for r in w.requests if r.stream < 8]
    go(warm, False)
    pool.sync()
    sat = go(w.requests, False)
    pool.sync()
    torch.cuda.synchronize()
    log(f"[bench] serving ({shape_name}) saturation: {sat.keys_per_s / 1e6:.1f} M keys/s, {sat.launches} launches, "
        f"{sat.mean_requests_per_launch:.1f} requests/launch, peak resident {sat.peak_resident}/{slots}")
    # the sampled streams against the oracle: each request is its own batch-schedule call
    import oracle
    verified = 0
    for st in check:
        ref = oracle.Sketch(shape["d"], shape["w"], shape["z"])
        for r in sorted((r for r in w.requests if r.stream == st), key=lambda r: r.seq):
            k = w.keys_of(r)
            if r.kind == sf.SF_REQ_QUERY:
                got = c_ans[(r.stream, r.seq)].cpu().numpy().view(np.uint32)
                if not np.array_equal(got, ref.query(k)):
                    raise SystemExit(f"serving ({shape_name}): stream {st} query {r.seq} differs from the oracle")
                verified += 1
            else:
                ops = np.full(r.n, 1 if r.kind == sf.SF_REQ_DELETE else 0, np.uint8)
                if ref.batch(k, ops, cfg.batch_ops, checked=True):
                    raise SystemExit("serving workload is not strict-turnstile")
        slim = c_slim[st].cpu().numpy().view(np.uint16).reshape(shape["d"], shape["w"])
        if not np.array_equal(slim, ref.slim()):
            raise SystemExit(f"serving ({shape_name}): stream {st}'s Slim differs from the oracle")
    log(f"[bench] serving ({shape_name}): streams {check} equal to the oracle ({verified} query answers, Slims)")
    span = max(r.arrival for r in w.requests)
    offered = total_keys / span
    import copy
    sweep = []
    for load in [float(x) for x in args.serve_loads.split(",") if x]:
        f = offered / (load * sat.keys_per_s)
        paced = [copy.copy(r) for r in w.requests]
        for r in paced:
            r.arrival *= f
        res = go(paced, True)
        pool.sync()
        sweep.append({"offered_load": load, "value": round(res.keys_per_s / 1e6, 2), "unit": "Mitems/s",
                      "latency_ms": res.latency_ms, "queueing_ms": res.queue_ms,
                      "latency_by_kind_ms": res.latency_by_kind_ms, "launches": res.launches,
                      "requests_per_launch": round(res.mean_requests_per_launch, 2),
                      "peak_resident_sketches": res.peak_resident})
        log(f"[bench] serving ({shape_name}) at {load:.2f} x saturation: {res.keys_per_s / 1e6:.1f} M keys/s, "
            f"latency {res.latency_ms}, by kind {res.latency_by_kind_ms}")
    pool.close()
    del joined
    torch.cuda.empty_cache()
    head = min(sweep, key=lambda x: abs(x["offered_load"] - 0.75)) if sweep else None
    out = {"workload": f"{w.n_streams} streams x 16 requests (insert/delete/query 0.7/0.1/0.2, "
                       "log-uniform 1K-1M uint32 keys, Zipf 1.0; deletes drawn uniformly from the stream's live "
                       f"occurrences), per-stream sketch d={shape['d']} Fat {shape['d']}x{shape['w'] * 4} u32, "
                       f"64 GiB HBM budget ({slots} resident sketches)",
           "saturation_mitems_s": round(sat.keys_per_s / 1e6, 2), "slots": slots,
           "owner_ratio": owner_ratio,
           "oracle_checked_streams": check, "oracle_checked_query_answers": verified, "sweep": sweep}
    if head:
        out.update({"offered_load": head["offered_load"], "value": head["value"], "unit": "Mitems/s",
                    "latency_ms": head["latency_ms"], "latency_by_kind_ms": head["latency_by_kind_ms"]})
    return out


def run_collector(np, sk, step, queries, answers, snapshots=20):
    """The Slim hand-off to a collector process (paper Sections 1 and 3): one
    snapshot after every update step (a reporting interval of one step), then
    back-to-back snapshots for the streaming rate, then the step's queries
    answered by the collector, which must equal the sketch's own answers."""
    from paper_1701_04148_amd.collector import Collector
    t_start = time.perf_counter()
    with Collector(max_cells=sk.d * sk.w, frames=4) as col:
        t_ready = time.perf_counter() - t_start
        col.publish(0, sk)                      # warm-up: the collector's first device copy
        col.drain()
        col.clear_latencies()
        for _ in range(snapshots):
            step()
            col.publish(0, sk)
        col.drain()
        lat = col.latencies()
        t0 = time.perf_counter()
        for _ in range(snapshots):
            col.publish(0, sk)
        col.drain()
        el = time.perf_counter() - t0
        t1 = time.perf_counter()
        got, seq = col.query(0, queries)
        q_el = time.perf_counter() - t1
    if not np.array_equal(got, answers):
        raise SystemExit("collector answers differ from the sketch's own")
    slim_bytes = 2 * sk.d * sk.w
    e2e, exp = lat["end_to_end_ms"], lat["export_ms"]
    return {"slim_bytes": slim_bytes, "frames": 4, "snapshots": int(lat["snapshots"]),
            "export_ms_p50": round(float(np.percentile(exp, 50)), 3),
            "to_collector_gpu_ms_p50": round(float(np.percentile(e2e, 50)), 3),
            "to_collector_gpu_ms_p99": round(float(np.percentile(e2e, 99)), 3),
            "stream_snapshots_per_s": round(snapshots / el, 1),
            "stream_gb_s": round(snapshots * slim_bytes / el / 1e9, 2),
            "query_keys": int(queries.shape[0]), "query_round_trip_ms": round(q_el * 1e3, 2),
            "answers_equal_sketch": True, "collector_start_s": round(t_ready, 1),
            "note": "sf_export_slim into a shared-memory frame (D2H), message over a pipe, the "
                    "collector process copies it to its GPU; query keys and answers travel over the pipe"}


LEG_NAMES = ("main", "main_s0.6", "main_s1.4", "small", "flows")
MERGE_PATHS = ("tile", "batch, owner for batches >= w", "batch+atomic", "batch+owner always")


def leg_workload(leg: str, sfgen, scale: int = 1):
    if leg == "small":
        return sfgen.config_small()
    if leg == "flows":
        return sfgen.config_flows(scale=scale)
    s = 1.0 if leg == "main" else float(leg.split("_s")[1])
    return sfgen.config_main(s, scale=scale)


def leg_config(leg: str, wl, b: int, n_del: int) -> dict:
    kind = "uint32" if wl.key_bytes == 4 else "13-byte flow"
    ops = (f"{wl.n_ops} {kind} ops Zipf(s={wl.meta['s']}) over {wl.meta['n_universe']} keys"
           + (f" with {n_del} deletes" if n_del else ", insert-only"))
    return {"workload": f"one SF-sketch d={wl.d}, Fat {wl.d}x{wl.w * wl.z} u32 (w={wl.w}, z={wl.z}), "
                        f"Slim {wl.d}x{wl.w} u16; {ops}; export Slim; {wl.n_queries} queries "
                        "(present + absent); keys resident in HBM",
            "sketches": 1, "d": wl.d, "w": wl.w, "z": wl.z, "key_bytes": wl.key_bytes, "ops": wl.n_ops,
            "deletes": n_del, "queries": wl.n_queries, "zipf_s": wl.meta["s"], "batch_ops": b}


def gpu_leg(args, torch, np, sf, wl, b: int, leg: str, steps: int, warmup: int) -> dict:
    """Times one single-sketch workload (reset, updates, Slim export, queries per step),
    then the same steps with per-kernel events; returns the numbers, the answers and the
    live sketch (for the host-fed and collector runs of the headline)."""
    dev = torch.device("cuda:0")
    kb = wl.key_bytes

    def dev_keys(a):
        if kb == 4:
            return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)
        return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(dev)

    keys = dev_keys(wl.keys)
    ops = torch.from_numpy(wl.ops).to(dev) if wl.ops is not None else None
    qk = dev_keys(wl.queries)
    out = torch.empty(wl.n_queries, dtype=torch.int32, device=dev)
    cells = wl.d * wl.w
    slim16 = torch.empty(cells, dtype=torch.int16, device=dev)
    n_del = int(wl.ops.sum()) if wl.ops is not None else 0
    n_ins = wl.n_ops - n_del
    sk = sf.Sketch(wl.d, wl.w, wl.z, key_bytes=kb, batch_ops=b)
    sk.set_tile(args.tile)
    sk.set_merge({"batch": 1, "atomic": 2, "owner": 3, "tile": 0}[args.merge])
    sk.set_streams({"auto": -1, "one": 0, "two": 1}[args.streams])
    if args.owner_range and sk.owner_range():
        try:
            sk.set_owner_range(args.owner_range)
        except sf.SFError as e:
            log(f"[bench] {leg}: owner range 2^{args.owner_range} not allowed for this shape ({e}); default kept")

    def step():
        sk.reset()
        if ops is None:
            sk.insert(keys)
        else:
            sk.update(keys, ops)
        sf.sf_export_slim(sk._h, slim16)
        sk.query(qk, out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ie0, de0 = sk.merge_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ie1, de1 = sk.merge_stats()
    ms_step = elapsed * 1e3 / steps
    value = (wl.n_ops + wl.n_queries) * steps / elapsed / 1e6
    log(f"[bench] {leg}: {steps} steps: {ms_step:.3f} ms/step, {value:.1f} M items/s")
    # Per-kernel durations: the same steps again with a HIP event pair around every
    # kernel group on the sketch's stream (the events add a gap after each group, so
    # these steps are not the timed ones).
    sk.profile(True)
    sk.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof_ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = sk.profile_read(reset=True)
    sk.profile(False)
    fat = sk.export_fat()
    rows = fat.reshape(wl.d, -1).astype(np.int64).sum(axis=1)
    if not (rows == n_ins - n_del).all():       # Section 3.4: every Fat row sums to the net weight
        raise SystemExit(f"{leg}: Fat row sums {rows} != net weight {n_ins - n_del}")
    answers = out.cpu().numpy().view(np.uint32).copy()
    u = dict(ins=n_ins * steps, dels=n_del * steps, ops=wl.n_ops * steps, q=wl.n_queries * steps,
             cells=cells * steps, mixed=ops is not None,
             ie=(ie1 - ie0) if args.merge != "tile" else n_ins * steps,
             de=(de1 - de0) if args.merge != "tile" else n_del * steps)
    kernels = {}
    for kind, (ms, launches, _) in prof.items():
        if not launches:
            continue
        byt = algorithmic_bytes(kind, wl.d, u, kb)
        acc = random_accesses(kind, wl.d, u)
        kernels[kind] = dict(ms_total=round(ms, 3), launches=launches, avg_launch_us=round(ms * 1e3 / launches, 2),
                             alg_gbs=round(byt / (ms * 1e-3) / 1e9, 1) if byt else None,
                             g_accesses_s=round(acc / (ms * 1e-3) / 1e9, 2) if acc else None)
    return dict(leg=leg, sk=sk, keys=keys, ops=ops, qk=qk, out=out, slim16=slim16, step=step,
                ms_step=ms_step, value=value, prof_ms=prof_ms, kernels=kernels, units=u, answers=answers,
                n_ins=n_ins, n_del=n_del, entries_per_step=[u["ie"] // steps, u["de"] // steps])


def roofline_of(g: dict, wl, b: int, scale: int) -> dict:
    """The dominant kernel's roofline: the owner step (k_own_step: its per-batch launches
    and the closing launch of each update call), or the largest kind on another path."""
    k, u, kb = g["kernels"], g["units"], g["wl_kb"]
    if "own_step" in k:
        kinds = [x for x in ("own_step", "own_final") if x in k]
        ms = sum(k[x]["ms_total"] for x in kinds)
        launches = sum(k[x]["launches"] for x in kinds)
        name, kind_for_traffic = "k_own_step", "own_step"
        alg = algorithmic_bytes("own_step", wl.d, u, kb)
    else:
        dom = max(k, key=lambda x: k[x]["ms_total"])
        ms, launches, name, kind_for_traffic = k[dom]["ms_total"], k[dom]["launches"], dom, dom
        alg = algorithmic_bytes(dom, wl.d, u, kb)
    avg_us = ms * 1e3 / launches
    achieved = alg / launches / (avg_us * 1e-6) / 1e9
    roof = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(kind_for_traffic, workload_tag(g["leg"], b, scale)),
            "avg_launch_us": round(avg_us, 2), "launches_per_step": round(launches / (u["ops"] / wl.n_ops), 2),
            "alg_bytes_per_launch": int(alg / launches)}
    if name == "k_own_step":
        rec_bytes = wl.d * wl.w * (wl.z + 1) * 4
        roof["streamed"] = {
            "what": "each launch reads its ranges' cell records into LDS and writes them back: at most "
                    "2 x the record array per launch",
            "bytes_per_launch_max": 2 * rec_bytes,
            "gbs_max": round(2 * rec_bytes / (avg_us * 1e-6) / 1e9, 1),
            "frac_max": round(2 * rec_bytes / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        if roof["traffic"]:
            roof["traffic_gbs"] = round(roof["traffic"] / (avg_us * 1e-6) / 1e9, 1)
            roof["traffic_frac"] = round(roof["traffic"] / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    return roof


def oracle_check(np, wl, b: int, gpu_answers, time_seq: bool = True, time_queries: bool = False) -> dict:
    """CPU oracle on the full workload: batch schedule (its answers must equal the GPU's
    bit for bit), strict sequential SF_F (accuracy against it), and optionally the
    queries on one core and on all cores.  Each oracle run is one thread."""
    import oracle
    from oracle import accuracy
    kb = wl.key_bytes
    runs = accuracy.run_modes(wl.d, wl.w, wl.z, kb, wl.keys, wl.ops, wl.queries, b,
                              modes=("seq", "batch") if time_seq else ("batch",))
    sk_b, ans_b, t_b = runs["batch"]                  # t_b: the updates alone
    parity = bool(np.array_equal(ans_b, gpu_answers))
    t0 = time.perf_counter()
    sk_b.query(wl.queries)
    t_q = time.perf_counter() - t0
    rep = {"parity_full_size": parity}
    items = wl.n_ops + wl.n_queries
    rep["cpu_baseline"] = {"value": round(items / (t_b + t_q) / 1e6, 3), "unit": "Mitems/s", "cores": 1,
                           "kind": "oracle",
                           "sample": f"the full workload ({wl.n_ops} ops + {wl.n_queries} queries), batch "
                                     f"schedule b={b}: updates {t_b:.1f}s + queries {t_q:.1f}s on 1 thread",
                           "batch_updates_mops": round(wl.n_ops / t_b / 1e6, 3)}
    if time_seq:
        _, _, t_s = runs["seq"]
        rep["cpu_baseline"]["seq_updates_mops"] = round(wl.n_ops / t_s / 1e6, 3)
        rep["cpu_baseline"]["seq_s"] = round(t_s, 2)
        rep["accuracy"] = accuracy.report(wl.d, wl.w, wl.z, kb, wl.keys, wl.ops, wl.queries, b, runs=runs)
    if time_queries:
        import threading
        info = cpu_info()
        nth = info["threads_for_all_cores"]
        q = wl.queries
        reps = max(1, (1 << 24) // max(1, q.shape[0]))        # about 16M queries per timing
        qq = np.concatenate([q] * reps) if reps > 1 else q
        t0 = time.perf_counter()
        sk_b.query(qq)
        t1 = time.perf_counter() - t0
        parts = np.array_split(np.arange(qq.shape[0]), nth)
        th = [threading.Thread(target=sk_b.query, args=(qq[p[0]:p[-1] + 1],)) for p in parts if p.size]
        t0 = time.perf_counter()
        for t in th:
            t.start()
        for t in th:
            t.join()
        tn = time.perf_counter() - t0
        rep["cpu_baseline"].update({
            "queries_1core_mqps": round(qq.shape[0] / t1 / 1e6, 2),
            "queries_all_cores_mqps": round(qq.shape[0] / tn / 1e6, 2),
            "query_threads": len(th), **info})
    return rep


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--legs", default=",".join(LEG_NAMES),
                    help="single-sketch legs to run, comma-separated (main first: it is the headline)")
    ap.add_argument("--batch-ops", type=int, default=0,
                    help="schedule batch size b of the headline (default: min(16 w, 2^23), the accuracy-backed rule)")
    ap.add_argument("--scale", type=int, default=1, help="divide the 32M-op and flow sizes (quick runs)")
    ap.add_argument("--tile", type=int, default=2048, help="ops per duplicate-merging tile (per-tile path)")
    ap.add_argument("--merge", choices=("tile", "batch", "atomic", "owner"), default="batch",
                    help="batch: batch-wide merge + owner-computes S1..S5 for batches of at least w ops; "
                         "atomic: batch-wide merge + atomic S1..S5; owner: owner-computes for every batch; "
                         "tile: per-tile merging")
    ap.add_argument("--no-lone-compare", action="store_true",
                    help="1024-sketch leg: skip the one-sketch-per-launch comparison (profiling runs)")
    ap.add_argument("--multi-shape-out", default="", help="write the 1024-sketch leg's batch sizes and group shape")
    ap.add_argument("--multi-shape-in", default="", help="run the 1024-sketch leg with a shape written before")
    ap.add_argument("--pool-owner-ratio", type=float, default=0.5,
                    help="serving pools: request batches of at least ratio * w ops take the owner path")
    ap.add_argument("--group-owner-ratio", type=float, default=0.0,
                    help="1024-sketch leg without autotuning: sf_group_set_owner_ratio")
    ap.add_argument("--group-round-ops", type=int, default=0,
                    help="ops per launch round of the 1024-sketch group (0: the library's default)")
    ap.add_argument("--owner-range", type=int, default=0,
                    help="owner path: ranges of 2^N cells (sf_set_owner_range; 0: the library's default)")
    ap.add_argument("--streams", choices=("auto", "one", "two"), default="auto",
                    help="owner path: partition of the next batch on a second stream (sf_set_streams)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain copy of this many MiB (known traffic, for byte counters)")
    ap.add_argument("--workload", choices=("main", "multi", "serve"), default="main",
                    help="main: the single-sketch legs (plus the multi and serve summaries unless "
                         "--no-multi / --no-serve); multi: 1024 sketches in one group; serve: the "
                         "request loop alone")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--no-host-fed", action="store_true", help="skip the PCIe-inclusive host-fed steps")
    ap.add_argument("--no-query-pipeline", action="store_true", help="skip the host-fed query batches")
    ap.add_argument("--no-collector", action="store_true",
                    help="skip streaming the Slim to a collector process")
    ap.add_argument("--no-autotune", action="store_true",
                    help="1024-sketch run: use the rule min(16 w, 2^23) instead of tuning b per width")
    ap.add_argument("--gen-workers", type=int, default=0,
                    help="processes generating the 1024-sketch streams (0: up to 16; 1 under a profiler)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-shape", choices=tuple(SERVE_SHAPES) + ("both",), default="both",
                    help="per-stream sketch: flows (d=8, the flow configuration; admission binds), "
                         "small (d=4, Fat 4 x 2^20; every stream fits) or both")
    ap.add_argument("--serve-loads", default="0.25,0.5,0.75,0.9",
                    help="offered loads (fractions of the measured saturation) the arrivals are replayed at")
    ap.add_argument("--serve-launch-keys", type=int, default=1 << 24)
    ap.add_argument("--stats-summary", metavar="STATS_CSV",
                    help="print a rocprofv3 --stats kernel table and exit")
    ap.add_argument("--trace-summary", metavar="TRACE_CSV",
                    help="print per-kind durations from a rocprofv3 kernel trace and exit")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="add one leg's PMC traffic (two rocprofv3 --pmc runs) to profiles/pmc_traffic.json "
                         "and exit; the leg is the first of --legs")
    ap.add_argument("--pmc-out", default="", help="PMC summary file to add to (default profiles/pmc_traffic.json)")
    args = ap.parse_args()
    legs = [x for x in args.legs.split(",") if x]
    for x in legs:
        if x not in LEG_NAMES:
            raise SystemExit(f"unknown leg {x}; choose from {LEG_NAMES}")

    def b_of(leg, w):
        if leg == "main" and args.batch_ops:
            return args.batch_ops
        return batch_for_width(w)

    if args.stats_summary:
        print(summarize_stats(args.stats_summary))
        return
    if args.trace_summary:
        print(summarize_trace(args.trace_summary))
        return
    if args.pmc_summary:
        import sfgen
        leg = legs[0]
        w = {"small": 16384, "flows": 2**21 // args.scale}.get(leg, 2**20 // args.scale)
        rec = summarize_pmc(args.pmc_summary[0], args.pmc_summary[1], workload_tag(leg, b_of(leg, w), args.scale),
                            args.copy_calibration_mib << 20)
        store_pmc(rec, args.pmc_out)
        print(format_pmc(rec))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1701_04148_amd as sf
    import sfgen

    if args.workload == "multi":
        print(json.dumps(run_multi(args, torch, np, sf, sfgen)), flush=True)
        return
    if args.workload == "serve":
        shapes = ("flows", "small") if args.serve_shape == "both" else (args.serve_shape,)
        w = serve_workload(args, sfgen)
        print(json.dumps({sh: run_serve(args, torch, np, sf, sfgen, sh, w) for sh in shapes}), flush=True)
        return

    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max_workers=max(1, min(8, cpu_info()["threads_for_all_cores"] // 2)))
    if args.copy_calibration_mib:
        from paper_1701_04148_amd import micro
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        micro.copy(src, dst, nb)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] calibration copy of {nb} bytes done")

    result, leg_out, jobs = None, {}, {}
    for leg in legs:
        t_gen = time.time()
        wl = leg_workload(leg, sfgen, args.scale)
        b = b_of(leg, wl.w)
        log(f"[bench] leg {leg}: workload {wl.name}: {wl.n_ops} ops, {wl.n_queries} queries, b={b}, "
            f"generated in {time.time() - t_gen:.1f}s")
        g = gpu_leg(args, torch, np, sf, wl, b, leg, args.steps, args.warmup)
        g["wl_kb"] = wl.key_bytes
        roof = roofline_of(g, wl, b, args.scale)
        step_bytes = step_algorithmic_bytes(wl.d, g["n_ins"], g["n_del"], wl.n_queries, wl.key_bytes)
        rec = {"value": round(g["value"], 2), "unit": "Mitems/s", "ms_per_step": round(g["ms_step"], 3),
               "config": leg_config(leg, wl, b, g["n_del"]), "roofline": roof,
               "step_roofline": {"achieved": round(step_bytes / (g["ms_step"] * 1e-3) / 1e9, 1), "unit": "GB/s",
                                 "peak": HBM_PEAK_GBS,
                                 "frac": round(step_bytes / (g["ms_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "bytes_per_step": step_bytes, "merged_entries_per_step": g["entries_per_step"]},
               "kernels": g["kernels"], "profiled_ms_per_step": round(g["prof_ms"], 3),
               "merge_path": MERGE_PATHS[g["sk"].merge_path()], "owner_range_shift": g["sk"].owner_range()}
        log(f"[bench] {leg}: roofline {json.dumps(roof)}")
        if leg == "main":
            result = {
                "metric": METRIC, "value": rec["value"], "unit": "Mitems/s", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
                "data": "synthetic", "config": rec["config"], "roofline": roof,
                "step_roofline": rec["step_roofline"], "kernels": g["kernels"],
                "kernels_note": "HIP-event durations from the same steps run once more with events on",
                "profiled_ms_per_step": rec["profiled_ms_per_step"], "merge_path": rec["merge_path"],
                "owner_range_shift": rec["owner_range_shift"],
                "phases_ms_per_step": {
                    "update": round(sum(v["ms_total"] for k, v in g["kernels"].items()
                                        if k not in ("query", "export")) / args.steps, 3),
                    "export": round(g["kernels"].get("export", {}).get("ms_total", 0.0) / args.steps, 3),
                    "query": round(g["kernels"].get("query", {}).get("ms_total", 0.0) / args.steps, 3)}}
            if not args.no_cpu_baseline:
                # the headline's CPU baseline alone on the host: batch and sequential updates on
                # one core, queries on one core and on all cores
                log("[bench] CPU oracle on the headline workload (1 thread per mode) ...")
                orc = oracle_check(np, wl, b, g["answers"], time_seq=True, time_queries=True)
                log(f"[bench] oracle: {json.dumps(orc['cpu_baseline'])}; parity {orc['parity_full_size']}")
                if not orc["parity_full_size"]:
                    raise SystemExit("GPU query answers differ from the oracle at full size")
                result["cpu_baseline"] = orc["cpu_baseline"]
                result["accuracy"] = orc["accuracy"]
                result["parity_full_size"] = True
            sk = g["sk"]
            if not args.no_host_fed and wl.ops is not None:
                result["host_fed"] = run_host_fed(torch, np, sf, g, wl, b, args.steps)
            if not args.no_query_pipeline:
                result["query_pipeline"] = run_query_pipeline(torch, np, g, wl)
            if not args.no_collector:
                result["collector"] = run_collector(np, sk, g["step"], wl.queries, g["answers"])
                log(f"[bench] collector: {json.dumps(result['collector'])}")
            if not args.no_autotune and wl.ops is not None:
                from paper_1701_04148_amd.tune import tune_batch
                t_tune = time.time()
                # the bound from the oracle's sequential ARE when the CPU leg has run
                seq_are = result.get("accuracy", {}).get("seq", {}).get("are")
                r = tune_batch(wl.d, wl.w, wl.z, wl.keys, wl.ops, wl.queries, modes=(2, 3), ref_are=seq_are,
                               shifts=None)
                result["autotune_check"] = {
                    "b": r.b, "merge_path": MERGE_PATHS[r.mode], "owner_range_shift": r.shift, "rule_b": b,
                    "ref": "oracle sequential SF_F" if seq_are is not None else f"GPU at b = {r.ref_b}",
                    "ref_are": round(r.ref_are, 5), "bound": round(r.bound, 5),
                    "candidates": [[bb, round(a, 5), round(ms, 2), ok, MERGE_PATHS[m], sh]
                                   for bb, a, ms, ok, m, sh in r.table]}
                log(f"[bench] autotuner on this workload ({time.time() - t_tune:.1f}s): b = {r.b}, "
                    f"path {result['autotune_check']['merge_path']}, range shift {r.shift} (rule {b})")
        else:
            leg_out[leg] = rec
            if not args.no_cpu_baseline:
                jobs[leg] = pool.submit(oracle_check, np, wl, b, g["answers"], True, False)
        g["sk"].close()
        del g
        torch.cuda.empty_cache()

    if result is None:      # the headline leg was not asked for: report the first leg as the line
        first = legs[0]
        rec = leg_out[first]
        result = {"metric": METRIC, "value": rec["value"], "unit": "Mitems/s", "n_gpus": 1, "steps": args.steps,
                  "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True,
                  "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
                  "config": rec["config"], "roofline": rec["roofline"], "kernels": rec["kernels"]}

    if not args.no_micro:
        log("[bench] random-access ceilings ...")
        result["random_access_ceilings_g_per_s"] = micro_ceilings(torch)
        log(f"[bench] ceilings {json.dumps(result['random_access_ceilings_g_per_s'])}")

    if not args.no_multi:
        multi = run_multi(args, torch, np, sf, sfgen)
        result["sketches_1024"] = {k: multi[k] for k in ("value", "unit", "ms_per_step", "config",
                                                         "one_sketch_per_launch", "group_vs_lone")}
        if multi.get("autotune"):
            result["sketches_1024"]["autotuned_b"] = {w: v["b"] for w, v in multi["autotune"].items()}
        if multi.get("group_shape"):
            result["sketches_1024"]["group_shape"] = multi["group_shape"]
        result["sketches_1024"]["kernels"] = multi["kernels"]
        if "cpu_baseline" in multi:
            result["sketches_1024"]["cpu_baseline"] = multi["cpu_baseline"]
        torch.cuda.empty_cache()
    # the legs' oracle runs end before the serving loop starts: its host-side
    # request loop then has the host to itself
    for leg, fut in jobs.items():
        log(f"[bench] waiting for the oracle of leg {leg} ...")
        orc = fut.result()
        if not orc["parity_full_size"]:
            raise SystemExit(f"{leg}: GPU query answers differ from the oracle at full size")
        cb = dict(orc["cpu_baseline"])
        cb["note"] = "timed while other legs ran on the GPU and other oracle runs shared the host"
        leg_out[leg].update(cpu_baseline=cb, accuracy=orc.get("accuracy"), parity_full_size=True)
        log(f"[bench] {leg}: oracle {json.dumps(cb)}")
    pool.shutdown()

    if not args.no_serve:
        w = serve_workload(args, sfgen)
        shapes = ("flows", "small") if args.serve_shape == "both" else (args.serve_shape,)
        for sh in shapes:
            result["serving" if sh == "flows" else f"serving_{sh}"] = run_serve(args, torch, np, sf, sfgen, sh, w)
    if leg_out:
        result["legs"] = leg_out
    print(json.dumps(result), flush=True)


def run_query_pipeline(torch, np, g, wl, batches=(20_000, 64_000, 256_000, 2_000_000), streams=(1, 4),
                       reps: int = 20) -> dict:
    """Host-fed query batches through sf_query_host (the multi-stream pipeline of the
    paper's GPU implementation): keys in pinned host memory, answers back in pinned
    host memory, per batch size and stream count: the median call latency and the
    query rate it gives.  The sketch holds the state of the last timed step (Slim
    exported); answers are checked against the device query of the same keys."""
    sk = g["sk"]
    q = wl.queries
    ref = g["answers"]
    rows = []
    for n in batches:
        n = min(n, q.shape[0])
        hk = torch.from_numpy(np.ascontiguousarray(q[:n]).view(np.int32)).pin_memory()
        out = torch.empty(n, dtype=torch.int32).pin_memory()
        for st in streams:
            sk.query_host(hk, out, streams=st)           # warm-up (buffers allocated)
            lat = []
            for _ in range(reps):
                t0 = time.perf_counter()
                sk.query_host(hk, out, streams=st)
                lat.append(time.perf_counter() - t0)
            if not np.array_equal(out.numpy().view(np.uint32), ref[:n]):
                raise SystemExit("sf_query_host answers differ from the device query")
            med = float(np.median(lat))
            rows.append({"batch": n, "streams": st, "latency_us_p50": round(med * 1e6, 1),
                         "latency_us_p99": round(float(np.percentile(lat, 99)) * 1e6, 1),
                         "mqps": round(n / med / 1e6, 2)})
    log(f"[bench] host-fed query pipeline: {json.dumps(rows)}")
    return {"rows": rows, "note": "keys H2D from pinned memory, query kernel, answers D2H, split over HIP "
                                  "streams (the first n mod streams take one more key); call latency includes "
                                  "the host-side launch and the wait for the last copy"}


def run_host_fed(torch, np, sf, g, wl, b: int, steps: int) -> dict:
    """PCIe-inclusive variant (never `value`): keys and op codes from pinned host memory
    through sf_update_host (copies overlap the updates), query keys copied in and answers
    copied out every step."""
    sk, qk, out, slim16 = g["sk"], g["qk"], g["out"], g["slim16"]
    hk = torch.from_numpy(wl.keys.view(np.int32)).pin_memory()
    ho = torch.from_numpy(wl.ops).pin_memory()
    hq = torch.from_numpy(wl.queries.view(np.int32)).pin_memory()
    hout = torch.empty(wl.n_queries, dtype=torch.int32).pin_memory()

    def host_step():
        sk.reset()
        sk.update_host(hk, ho, chunk_ops=b)
        sf.sf_export_slim(sk._h, slim16)
        qk.copy_(hq, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        sk.query(qk, out)
        sk.sync()
        hout.copy_(out)

    host_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        host_step()
    torch.cuda.synchronize()
    hel = time.perf_counter() - t0
    items = (wl.n_ops + wl.n_queries) * steps
    rec = {"value": round(items / hel / 1e6, 2), "unit": "Mitems/s", "ms_per_step": round(hel * 1e3 / steps, 3),
           "note": "keys + op codes + query keys H2D from pinned memory and answers D2H "
                   "each step (sf_update_host, copy chunks of b ops overlapping the updates)"}
    log(f"[bench] host-fed (PCIe-inclusive): {rec['ms_per_step']} ms/step, {rec['value']} M items/s")
    return rec


if __name__ == "__main__":
    main()
