#!/usr/bin/env python3
"""SF-sketch hot-path benchmark on one MI355X.

One step = the whole hot path over one batch of synthetic input, with keys
already resident in HBM: re-zero the sketch, apply the op stream (inserts and
deletes through the deterministic batch schedule), export the Slim (what the
monitor ships to the collector), and answer the point queries.

Default workload: one SF-sketch, d=4, Fat 4 x 2^22 uint32 (w=2^20 buckets of
z=4), Slim 4 x 2^20 uint16; 32M uint32 ops, Zipf(s=1.0) over 1M distinct
keys, 10% deletions of live occurrences; queries = the 1M keys + 1M absent.

Prints ONE JSON line (rank 0): throughput in M items/s (ops + queries), the
dominant kernel's roofline object, and the CPU oracle timed on the host.
Progress goes to stderr.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    """Digest of the kernel sources; a stored counter reading is valid only for it."""
    h = hashlib.sha256()
    for rel in ("paper_1701_04148_amd/csrc/sf_lib.hip", "paper_1701_04148_amd/csrc/sf_device.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kind: str, d: int, n_ins: int, n_del: int, n_ops: int, mixed: bool,
                      n_q: int, cells: int) -> int:
    """Bytes a kernel's step must move, each access counted at its element size
    (uint32 key, uint32 Slim working cell, uint32 Fat counter, 16 B Fat bucket,
    the snapshot the batch schedule defines, 1 B op code when ops are mixed)."""
    op_byte = n_ops if mixed else 0
    if kind == "snapshot":   # key, Slim cell, Fat counter; snapshot write 4 + 2 B per row
        return n_ins * (4 + d * (4 + 4 + 4 + 2)) + op_byte
    if kind == "fat_add":    # key, Fat read-modify-write
        return n_ins * (4 + d * 8) + op_byte
    if kind == "raise":      # key, Fat counter, snapshot read 4 + 2 B per row
        return n_ins * (4 + d * (4 + 4 + 2)) + op_byte
    if kind == "fat_sub":
        return n_del * (4 + d * 8) + op_byte
    if kind == "clamp":      # key, 16-B bucket, Slim cell
        return n_del * (4 + d * (16 + 4)) + op_byte
    if kind == "query":      # key, d Slim cells, answer
        return n_q * (4 + d * 4 + 4)
    if kind == "export":     # uint32 working cell in, uint16 out
        return cells * 6
    return 0


# random accesses per unit of each kernel (reads + atomics, merged duplicates not subtracted)
def random_accesses(kind: str, d: int, n_ins: int, n_del: int, n_q: int) -> int:
    return {"snapshot": 2 * d * n_ins, "fat_add": d * n_ins, "raise": d * n_ins,
            "fat_sub": d * n_del, "clamp": 2 * d * n_del, "query": d * n_q}.get(kind, 0)


def stored_traffic(kernel_kind: str, workload: str):
    """HBM bytes per launch from the committed PMC summary, if taken on these sources."""
    path = os.path.join(PROFILE_DIR, "pmc_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest() or rec.get("workload") != workload:
        return None
    k = rec.get("kernels", {}).get(kernel_kind)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


KIND_OF_KERNEL = {"k_snapshot": "snapshot", "k_raise": "raise", "k_clamp": "clamp",
                  "k_query": "query", "k_pack16": "export"}


def _kernel_base(name: str) -> str:
    base = name.replace("(anonymous namespace)::", "").replace("void ", "").strip()
    return base.split("(")[0].split("<")[0].strip()


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
            if base == "k_fat_update":
                kind = "fat_sub" if prev == "k_raise" else "fat_add"
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


def workload_tag(args) -> str:
    """Name of the timed workload (sketch shape, stream, schedule, tile) for stored counters."""
    return (f"c2_d4_w{2**20 // args.scale}_z4_ops{32_000_000 // args.scale}_zipf{args.skew}_del10"
            f"_b{args.batch_ops}_tile{args.tile}")


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
                         ("pair_two_lines", lambda s: micro.gather_pair(t, n, s, False, sink))):
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--skew", type=float, default=1.0, help="Zipf s (0.6, 1.0, 1.4)")
    ap.add_argument("--batch-ops", type=int, default=1 << 21, help="schedule batch size b")
    ap.add_argument("--scale", type=int, default=1, help="divide every size (quick runs)")
    ap.add_argument("--tile", type=int, default=2048, help="ops per duplicate-merging tile")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain copy of this many MiB (known traffic, for byte counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/pmc_traffic.json from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()

    if args.pmc_summary:
        rec = summarize_pmc(args.pmc_summary[0], args.pmc_summary[1], workload_tag(args),
                            args.copy_calibration_mib << 20)
        with open(os.path.join(PROFILE_DIR, "pmc_traffic.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1701_04148_amd as sf
    import sfgen

    t_gen = time.time()
    wl = sfgen.config_main(args.skew, scale=args.scale)
    log(f"[bench] workload {wl.name}: {wl.n_ops} ops ({int(wl.ops.sum())} deletes), "
        f"{wl.n_queries} queries, generated in {time.time() - t_gen:.1f}s")
    n_del = int(wl.ops.sum())
    n_ins = wl.n_ops - n_del
    cells = wl.d * wl.w
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(wl.keys.view(np.int32)).to(dev)
    ops = torch.from_numpy(wl.ops).to(dev)
    qk = torch.from_numpy(wl.queries.view(np.int32)).to(dev)
    out = torch.empty(wl.n_queries, dtype=torch.int32, device=dev)
    slim16 = torch.empty(cells, dtype=torch.int16, device=dev)
    b = args.batch_ops
    sk = sf.Sketch(wl.d, wl.w, wl.z, batch_ops=b)
    sk.set_tile(args.tile)

    def step():
        sk.reset()
        sk.update(keys, ops)
        sf.sf_export_slim(sk._h, slim16)
        sk.query(qk, out)

    if args.copy_calibration_mib:
        from paper_1701_04148_amd import micro
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        micro.copy(src, dst, nb)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] calibration copy of {nb} bytes done")
    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")
    sk.profile(True)
    sk.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = sk.profile_read(reset=True)
    sk.profile(False)
    ms_step = elapsed * 1e3 / args.steps
    items = (wl.n_ops + wl.n_queries) * args.steps
    value = items / elapsed / 1e6
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step, {value:.1f} M items/s")

    # sanity on the device result: Fat row sums = net stream weight (Section 3.4 CM property)
    fat = sk.export_fat()
    rows = fat.reshape(wl.d, -1).astype(np.int64).sum(axis=1)
    if not (rows == n_ins - n_del).all():
        raise SystemExit(f"Fat row sums {rows} != net weight {n_ins - n_del}")
    gpu_answers = out.cpu().numpy().view(np.uint32).copy()

    # per-kernel accounting from the events on the sketch's stream
    kernels = {}
    for kind, (ms, launches, _) in prof.items():
        if not launches:
            continue
        byt = algorithmic_bytes(kind, wl.d, n_ins, n_del, wl.n_ops, True, wl.n_queries, cells) * args.steps
        acc = random_accesses(kind, wl.d, n_ins, n_del, wl.n_queries) * args.steps
        kernels[kind] = dict(ms_total=round(ms, 3), launches=launches,
                             avg_launch_us=round(ms * 1e3 / launches, 2),
                             alg_gbs=round(byt / (ms * 1e-3) / 1e9, 1),
                             g_accesses_s=round(acc / (ms * 1e-3) / 1e9, 2) if acc else None)
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
    dk = kernels[dom]
    alg_per_launch = algorithmic_bytes(dom, wl.d, n_ins, n_del, wl.n_ops, True, wl.n_queries,
                                       cells) * args.steps / dk["launches"]
    achieved = alg_per_launch / (dk["avg_launch_us"] * 1e-6) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic(dom, workload_tag(args))}
    log(f"[bench] kernels: {json.dumps(kernels)}")

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mitems/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "one SF-sketch d=4, Fat 4x2^22 u32 (w=2^20, z=4), Slim 4x2^20 u16; "
                               f"{wl.n_ops} uint32 ops Zipf(s={args.skew}) over {wl.meta['n_universe']} keys "
                               f"with {n_del} deletes; export Slim; {wl.n_queries} queries "
                               "(present + absent); keys resident in HBM",
                   "sketches": 1, "d": wl.d, "w": wl.w, "z": wl.z, "ops": wl.n_ops, "deletes": n_del,
                   "queries": wl.n_queries, "zipf_s": args.skew, "batch_ops": b, "tile_ops": args.tile,
                   "scale": args.scale},
        "roofline": roofline,
        "kernels": kernels,
    }

    if not args.no_micro:
        log("[bench] random-access ceilings ...")
        ceil = micro_ceilings(torch)
        result["random_access_ceilings_g_per_s"] = ceil
        log(f"[bench] ceilings {json.dumps(ceil)}")

    if not args.no_cpu_baseline:
        import oracle
        log("[bench] CPU oracle (single thread, batch schedule, same inputs) ...")
        ref = oracle.Sketch(wl.d, wl.w, wl.z)
        c0 = time.perf_counter()
        rc = ref.batch(wl.keys, wl.ops, b)
        ans = ref.query(wl.queries)
        c_el = time.perf_counter() - c0
        if rc:
            raise SystemExit(f"oracle failed {rc}")
        result["cpu_baseline"] = {"value": round((wl.n_ops + wl.n_queries) / c_el / 1e6, 3),
                                  "unit": "Mitems/s", "cores": 1, "kind": "oracle",
                                  "sample": f"one full step of the same workload ({wl.n_ops} ops + "
                                            f"{wl.n_queries} queries), batch schedule b={b}, "
                                            f"{c_el:.1f}s on 1 thread"}
        result["parity_full_size"] = bool(np.array_equal(ans, gpu_answers))
        log(f"[bench] oracle {c_el:.1f}s; GPU answers bit-exact: {result['parity_full_size']}")
        if not result["parity_full_size"]:
            raise SystemExit("GPU query answers differ from the oracle at full size")

    sk.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
