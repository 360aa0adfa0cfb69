// libsf.so: sketch groups -- many independent SF-sketches (one per monitoring
// node, each with its own stream of ops) updated and queried together.
//
// Every sketch keeps its own schedule: its ops are cut into batches of its
// own batch_ops, exactly as a single sketch would cut them, so a group gives
// each sketch the same state it would reach alone.  Round k runs batch k of
// every sketch that has one.  Sketches are independent, so a round may be
// split into sub-rounds (each sketch's batch whole inside one) to bound the
// snapshot scratch; sub-round order does not matter.  Each sub-round is one
// launch of each schedule step over a device table of tiles (ListPlan); a
// whole update call can be captured into one hipGraph and replayed.
//
// By default a sub-round goes through the batch-merge path: its ops are
// partitioned into hash buckets of (key, sketch) pairs, merged in LDS into
// one entry per distinct pair and chunk, and S1..S5 run once per entry.
// Merged sub-rounds hold at most kMergeRound ops (or one sketch's batch, if
// larger): larger sub-rounds mean fewer launches, but past 2^24 ops the 512
// buckets per op type span several LDS chunks each and fewer duplicates merge.
// When every sketch has the same d and z, S1..S5 run owner-computes: each
// sub-round numbers its sketches' cell ranges in a table of its own, and one
// workgroup per (row, range) stages the range's records in LDS (sf_owner.hpp);
// a sketch whose batch is sparse for its width (owner ratio) keeps the atomic
// entry kernels in the same sub-round.
//
// Device memory: one allocation holds every sketch's cell records (Fat
// bucket and Slim working copy of a cell side by side), the sketch table,
// export staging (largest dense Fat), the snapshot scratch
// ([d_max][round_ops] uint32 + uint16) and the merge buffers (partitioned
// keys, entries, counts for one merged sub-round); the owner path's buffers
// are a second one, and the tile and range tables grow as needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "sf.h"
#include "sf_host.hpp"

using namespace sfk;
using namespace sfh;

struct sf_group {
    uint32_t n;
    uint32_t key_bytes;
    uint32_t d_max;
    uint32_t d_uniform;  // common d, or 0 when the sketches differ
    std::vector<sf_config> cfg;
    std::vector<SketchDesc> desc;  // host copy of the sketch table
    hipStream_t stream;
    bool own_stream;               // created here: graphs cannot capture the null stream
    char* base;                    // the one allocation
    uint64_t state_bytes;          // Fat + Slim region (zeroed by reset)
    SketchDesc* d_desc;
    uint16_t* stage;
    uint32_t* bpre;
    uint16_t* asnap;
    uint64_t round_ops;            // snapshot capacity in ops
    uint64_t merge_round;          // ops of a merged sub-round (<= round_ops)
    void* part;                    // merge buffers, merge_round entries each
    void* ent_key;
    uint32_t* ent_cnt;
    MergeMeta* meta;
    uint32_t* hist;                // per-group bucket histograms of a merged sub-round
    MergeChunk* chunks;            // key range of every merge chunk of a merged sub-round
    uint64_t hist_groups;          // partition groups (tiles) a merged sub-round may have
    uint32_t tile_j;
    bool use_graph;
    bool merge;                    // batch-merge path (default) or per-tile merging
    // owner-computes S1..S5 (batch-merge path, when every sketch has the same
    // d and z): buffers for one merged sub-round and each sub-round's ranges
    bool owner_ok = false;         // the shapes fit (buffers allocated)
    bool owner_on = false;         // merge mode 1
    double own_ratio = 0.0;        // a sketch's batch is owner-computed when its ops >= own_ratio * w
    OwnerGeom own_og{};            // cr_shift, zbits, d (R and ncol are per sub-round)
    OwnerBufs own{};
    char* own_base = nullptr;
    uint32_t* d_ranges = nullptr;  // per sub-round: qbase [n], then qsk and qr [Q each]
    size_t ranges_cap = 0;
    std::vector<uint32_t> h_ranges;
    uint64_t own_sizes[6] = {};    // pairs, pos, res, level, hmat, pair meta (bytes)
    // the last query call's table on the device (d_qtiles)
    const void* q_keys = nullptr;
    const uint32_t* q_out = nullptr;
    std::vector<uint64_t> q_seg;
    size_t q_tiles = 0;
    // tile table (device, growable) and its pinned host staging
    TileDesc* d_tiles = nullptr;
    size_t tiles_cap = 0;
    TileDesc* h_tiles = nullptr;
    size_t h_cap = 0;
    // the last update call's plan and its captured graph
    std::vector<TileDesc> plan;
    struct SubRound {
        uint32_t first, tiles;
        uint64_t ops;
        uint32_t ranges = 0;       // owner path: ranges per row (Q) of its owner-computed sketches
        uint64_t table = 0;        // owner path: offset of its range table in d_ranges (words)
        bool atomic_side = false;  // owner path: some of its sketches keep the atomic entry kernels
    };
    std::vector<SubRound> subrounds;
    uint32_t plan_kind = 0;
    bool plan_on_device = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // query tiles (device, growable)
    TileDesc* d_qtiles = nullptr;
    size_t qtiles_cap = 0;
    Profiler prof;
};

namespace {

std::mutex g_mu;
std::unordered_set<const sf_group*> g_live;

bool live(const sf_group* g) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g && g_live.count(g);
}

constexpr uint64_t kMergeRound = 1ull << 24;
constexpr uint64_t kHistExtra = 1024;  // partial tiles (one per sketch) a merged sub-round may add

struct Layout {
    std::vector<uint64_t> fat_off;  // each sketch's cell records (Fat bucket + Slim per cell)
    uint64_t state, desc, stage, bpre, asnap, part, ent_key, ent_cnt, meta, hist, chunks, total;
    uint64_t round_ops, merge_round;
    uint32_t d_max;
    bool owner = false;             // owner-computes buffers (a second allocation, counted in total)
    OwnerGeom og{};
    uint64_t pairs = 0, pos = 0, res = 0, level = 0, hmat = 0, pmeta = 0;
    uint64_t owner_bytes() const { return pairs + pos + res + level + hmat + pmeta; }
};

// Ranges per row one sub-round may hold: the pair kernels' tables, as far as
// the columns of both op types over d rows fit kMaxCols.  (Twice as many
// ranges per sub-round, in wider tables, measured slower: larger sub-rounds
// spread a bucket over more merge chunks, which merge fewer duplicates.)
inline uint32_t table_range_cap(uint32_t d) { return std::min<uint32_t>(kMaxRanges, kMaxCols / (2 * d)); }

// The owner path for a sketch table: every sketch with the same d and z;
// ranges of 2^k cells, k the largest with at most 8192 Fat counters per range
// (and a 16-bit local code), at most table_range_cap(d) per row in one
// sub-round.
bool group_owner_geom(uint32_t n, const sf_config* cfgs, OwnerGeom* og) {
    for (uint32_t i = 1; i < n; i++)
        if (cfgs[i].d != cfgs[0].d || cfgs[i].z != cfgs[0].z) return false;
    const uint32_t d = cfgs[0].d, z = cfgs[0].z;
    uint32_t zbits = 0;
    while ((1ull << zbits) < z) zbits++;
    uint32_t sh = 4;
    while ((2ull << sh) * z <= kOwnCounters && ((2ull << sh) << zbits) <= 65536) sh++;
    if ((1ull << sh) * z > kOwnCounters || ((1ull << sh) << zbits) > 65536) return false;
    for (uint32_t i = 0; i < n; i++)  // each sketch fits a sub-round on its own
        if (((uint64_t(cfgs[i].w) + (1ull << sh) - 1) >> sh) > table_range_cap(d)) return false;
    *og = OwnerGeom{};
    og->cr_shift = sh;
    og->zbits = zbits;
    og->d = d;
    return true;
}

int layout_of(uint32_t n, const sf_config* cfgs, uint64_t round_ops, Layout& L) {
    if (n == 0 || !cfgs) return fail(SF_EINVAL, "a group needs at least one sketch config");
    uint64_t off = 0, max_b = 0, max_stage = 0;
    L.d_max = 0;
    L.fat_off.resize(n);
    for (uint32_t i = 0; i < n; i++) {
        int rc = validate(&cfgs[i]);
        if (rc) return fail(rc, "sketch " + std::to_string(i) + ": " + last_error());
        if (cfgs[i].key_bytes != cfgs[0].key_bytes) return fail(SF_EINVAL, "key_bytes must match across a group");
        const uint64_t cells = uint64_t(cfgs[i].d) * cfgs[i].w;
        L.fat_off[i] = off;
        off += round256(cells * (cfgs[i].z + 1) * 4);
        max_b = std::max<uint64_t>(max_b, cfgs[i].batch_ops);
        max_stage = std::max<uint64_t>(max_stage, cells * cfgs[i].z * 4);  // dense Fat export
        L.d_max = std::max(L.d_max, cfgs[i].d);
    }
    L.state = off;
    if (round_ops == 0) {
        uint64_t sum_b = 0;
        for (uint32_t i = 0; i < n; i++) sum_b += cfgs[i].batch_ops;
        round_ops = std::min<uint64_t>(sum_b, 1ull << 26);
    }
    L.round_ops = std::max(round_ops, max_b);
    if (L.round_ops > (1ull << 31)) return fail(SF_EINVAL, "round_ops must be <= 2^31");
    L.desc = off;
    off += round256(uint64_t(n) * sizeof(SketchDesc));
    L.stage = off;
    off += round256(max_stage);
    L.bpre = off;
    off += round256(uint64_t(L.d_max) * L.round_ops * 4);
    L.asnap = off;
    off += round256(uint64_t(L.d_max) * L.round_ops * 2);
    L.merge_round = std::max(std::min(L.round_ops, kMergeRound), max_b);
    const uint64_t mkey = cfgs[0].key_bytes == 4 ? sizeof(MKey<4, true>) : sizeof(MKey<13, true>);
    L.part = off;
    off += round256(L.merge_round * mkey);
    L.ent_key = off;
    off += round256(L.merge_round * mkey);
    L.ent_cnt = off;
    off += round256(L.merge_round * 4);
    L.meta = off;
    off += round256(sizeof(MergeMeta));
    L.hist = off;
    off += round256(part_groups_max(L.merge_round, kHistExtra) * 2 * kMaxBuckets * 4);
    L.chunks = off;
    off += round256(merge_chunks_max(L.merge_round) * sizeof(MergeChunk));
    L.total = off;
    L.owner = group_owner_geom(n, cfgs, &L.og);
    if (L.owner) {
        const uint64_t mr = L.merge_round, d = L.og.d;
        L.pairs = round256(d * mr * 8);
        L.pos = round256(d * mr * 4);
        L.res = round256(d * mr * 8);
        L.level = round256(mr * 2);
        L.hmat = round256(uint64_t(pair_tiles_max(uint32_t(mr))) * 2 * d * table_range_cap(uint32_t(d)) * 4);
        L.pmeta = round256(sizeof(PairMeta));
        L.total += L.owner_bytes();
    }
    return SF_OK;
}

int ensure_device_tiles(TileDesc*& buf, size_t& cap, size_t need) {
    if (need <= cap) return SF_OK;
    size_t ncap = std::max<size_t>(need, cap * 2 + 1024);
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&buf), ncap * sizeof(TileDesc));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        buf = nullptr;
        return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "tile table") : device_fail(e, "tile table");
    }
    cap = ncap;
    return SF_OK;
}

int upload_tiles(sf_group* g, TileDesc* dst, const std::vector<TileDesc>& src) {
    if (src.empty()) return SF_OK;
    if (g->h_cap < src.size()) {
        if (g->h_tiles) (void)hipHostFree(g->h_tiles);
        g->h_tiles = nullptr;
        g->h_cap = 0;
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&g->h_tiles), src.size() * sizeof(TileDesc),
                                     hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return device_fail(e, "pinned tile staging");
        }
        g->h_cap = src.size();
    }
    std::memcpy(g->h_tiles, src.data(), src.size() * sizeof(TileDesc));
    hipError_t e = hipMemcpyAsync(dst, g->h_tiles, src.size() * sizeof(TileDesc), hipMemcpyHostToDevice,
                                  g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);  // staging reused by the next call
    return e == hipSuccess ? SF_OK : device_fail(e, "tile upload");
}

int check_segments(const sf_group* g, const uint64_t* seg) {
    if (!seg) return fail(SF_EINVAL, "seg is null");
    if (seg[0] != 0) return fail(SF_EINVAL, "seg[0] must be 0");
    for (uint32_t i = 0; i < g->n; i++)
        if (seg[i + 1] < seg[i]) return fail(SF_EINVAL, "seg must be non-decreasing");
    return SF_OK;
}

// Cut every sketch's ops into its own batches; round k = batch k of every
// sketch; rounds split into sub-rounds of at most round_ops ops (merged:
// merge_round ops, tiles of kPartOps ops for the partition kernels).
void build_plan(sf_group* g, const uint64_t* seg, const uint8_t* keys, const uint8_t* ops, uint32_t mode) {
    g->plan.clear();
    g->subrounds.clear();
    const bool owner = g->merge && g->owner_on;
    const uint32_t qcap = owner ? table_range_cap(g->own_og.d) : 0u;
    // the owner path streams every range of a sketch; a batch that touches its
    // sketch sparsely (fewer than own_ratio * w ops) keeps the atomic kernels
    auto owns = [&](uint32_t s, uint64_t cnt) {
        return owner && double(cnt) >= g->own_ratio * double(g->cfg[s].w);
    };
    auto ranges_of = [&](uint32_t s, uint64_t cnt) {
        return owns(s, cnt)
                   ? uint32_t((uint64_t(g->cfg[s].w) + (1ull << g->own_og.cr_shift) - 1) >> g->own_og.cr_shift)
                   : 0u;
    };
    const uint32_t tile_ops = g->merge ? kPartOps : uint32_t(kBlock) * g->tile_j;
    const uint64_t limit = g->merge ? g->merge_round : g->round_ops;
    const uint64_t max_tiles = g->merge ? g->hist_groups : ~0ull;
    uint64_t rounds = 0;
    for (uint32_t s = 0; s < g->n; s++) {
        const uint64_t len = seg[s + 1] - seg[s], b = g->cfg[s].batch_ops;
        rounds = std::max(rounds, (len + b - 1) / b);
    }
    for (uint64_t k = 0; k < rounds; k++) {
        uint64_t used = 0;
        uint32_t first = uint32_t(g->plan.size()), q = 0;
        bool side = false;
        for (uint32_t s = 0; s < g->n; s++) {
            const uint64_t b = g->cfg[s].batch_ops;
            const uint64_t lo = seg[s] + k * b;
            if (lo >= seg[s + 1]) continue;
            const uint64_t cnt = std::min(b, seg[s + 1] - lo);
            const uint64_t tiles = (cnt + tile_ops - 1) / tile_ops;
            if (used && (used + cnt > limit || g->plan.size() - first + tiles > max_tiles ||
                         q + ranges_of(s, cnt) > qcap)) {  // close the sub-round
                g->subrounds.push_back({first, uint32_t(g->plan.size()) - first, used, q, 0, side});
                first = uint32_t(g->plan.size());
                used = 0;
                q = 0;
                side = false;
            }
            q += ranges_of(s, cnt);
            side = side || (owner && !owns(s, cnt));
            for (uint64_t off = 0; off < cnt; off += tile_ops) {
                TileDesc t{};
                t.keys = keys + (lo + off) * g->key_bytes;
                t.ops = mode == kOpsArray ? ops + lo + off : nullptr;
                t.count = uint32_t(std::min<uint64_t>(tile_ops, cnt - off));
                t.sketch = s;
                t.scr = uint32_t(used + off);
                t.mode = mode;
                g->plan.push_back(t);
            }
            used += cnt;
        }
        if (uint32_t(g->plan.size()) > first)
            g->subrounds.push_back({first, uint32_t(g->plan.size()) - first, used, q, 0, side});
    }
    if (!owner) return;
    // each sub-round's range table: its sketches' ranges numbered in plan order
    g->h_ranges.clear();
    for (auto& sr : g->subrounds) {
        sr.table = g->h_ranges.size();
        g->h_ranges.resize(sr.table + g->n + 2ull * sr.ranges, ~0u);
        uint32_t* qbase = g->h_ranges.data() + sr.table;
        uint32_t* qsk = qbase + g->n;
        uint32_t* qr = qsk + sr.ranges;
        uint32_t qn = 0;
        for (uint32_t t = sr.first; t < sr.first + sr.tiles;) {
            const uint32_t s = g->plan[t].sketch;
            uint64_t cnt = 0;  // the sketch's batch: its consecutive tiles
            for (; t < sr.first + sr.tiles && g->plan[t].sketch == s; t++) cnt += g->plan[t].count;
            if (!owns(s, cnt)) continue;  // atomic path: no ranges (qbase stays ~0)
            qbase[s] = qn;
            for (uint32_t r = 0, nr = ranges_of(s, cnt); r < nr; r++, qn++) {
                qsk[qn] = s;
                qr[qn] = r;
            }
        }
    }
}

// The owner-path buffers (pairs, positions, snapshots, T, column counts),
// sized for one merged sub-round.
int group_owner_alloc(sf_group* g) {
    const uint64_t* sz = g->own_sizes;
    const uint64_t total = sz[0] + sz[1] + sz[2] + sz[3] + sz[4] + sz[5];
    char* ob = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&ob), total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "owner-path buffers: out of device memory")
                                        : device_fail(e, "owner-path buffers");
    }
    g->own_base = ob;
    g->own = OwnerBufs{};
    g->own.og = g->own_og;
    g->own.pairs[0] = reinterpret_cast<uint64_t*>(ob);
    g->own.pairs[1] = nullptr;
    g->own.pos = reinterpret_cast<uint32_t*>(ob + sz[0]);
    g->own.res = reinterpret_cast<uint64_t*>(ob + sz[0] + sz[1]);
    g->own.level = reinterpret_cast<uint16_t*>(ob + sz[0] + sz[1] + sz[2]);
    g->own.hmat = reinterpret_cast<uint32_t*>(ob + sz[0] + sz[1] + sz[2] + sz[3]);
    g->own.pm[0] = reinterpret_cast<PairMeta*>(ob + sz[0] + sz[1] + sz[2] + sz[3] + sz[4]);
    g->own.pm[1] = nullptr;
    g->owner_on = true;
    return SF_OK;
}

int upload_ranges(sf_group* g) {
    const size_t words = g->h_ranges.size();
    if (!words) return SF_OK;
    if (g->ranges_cap < words) {
        if (g->d_ranges) (void)hipFree(g->d_ranges);
        g->d_ranges = nullptr;
        g->ranges_cap = 0;
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&g->d_ranges), words * 4);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "range tables") : device_fail(e, "range tables");
        }
        g->ranges_cap = words;
    }
    hipError_t e = hipMemcpy(g->d_ranges, g->h_ranges.data(), words * 4, hipMemcpyHostToDevice);
    return e == hipSuccess ? SF_OK : device_fail(e, "range table upload");
}

template <int KB>
void launch_plan(sf_group* g, bool ins, bool del, Profiler* prof) {
    MergeRun<KB, true> run{static_cast<MKey<KB, true>*>(g->part), static_cast<MKey<KB, true>*>(g->ent_key),
                           g->ent_cnt, g->meta, g->hist, g->chunks, uint32_t(g->merge_round), g->bpre,
                           g->asnap,
                           uint32_t(g->round_ops)};
    const SketchTable table{g->d_desc};
    const bool owner = g->merge && g->owner_on;
    for (auto& sr : g->subrounds) {
        const ListPlan<KB> plan{g->d_tiles + sr.first, g->d_desc};
        const uint32_t cnt = uint32_t(sr.ops);
        run.own = nullptr;
        if (owner && sr.ranges) {
            run.own = &g->own;
            run.side_atomic = sr.atomic_side;
            run.sub_og = g->own_og;
            run.sub_og.R = sr.ranges;
            run.sub_og.ncol = 2 * g->own_og.d * sr.ranges;
            run.sub_og.xcd = (kXcds % g->own_og.d == 0 && (g->own_og.d * sr.ranges) % kXcds == 0) ? 1u : 0u;
            run.sub_rm = TableRanges{g->d_ranges + sr.table, g->d_ranges + sr.table + g->n,
                                     g->d_ranges + sr.table + g->n + sr.ranges};
            run.max_z = g->cfg[0].z;
        }
        if (!g->merge) {
            Steps<ListPlan>::by_rows<KB>(g->d_uniform, g->tile_j, plan, sr.tiles, ins, del, g->bpre, g->asnap,
                                        uint32_t(g->round_ops), g->stream, prof, cnt);
        } else if (g->d_uniform == 4) {
            run.template launch<4>(plan, sr.tiles, cnt, table, ins, del, g->stream, prof);
        } else if (g->d_uniform == 8) {
            run.template launch<8>(plan, sr.tiles, cnt, table, ins, del, g->stream, prof);
        } else {
            run.template launch<0>(plan, sr.tiles, cnt, table, ins, del, g->stream, prof);
        }
    }
}

void drop_graph(sf_group* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->exec = nullptr;
    g->graph = nullptr;
}

enum Kind : uint32_t { kInsert = 1, kDelete = 2, kMixed = 3 };

int group_updates(sf_group* g, const void* keys, const uint8_t* ops, const uint64_t* seg, Kind kind) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    int rc = check_segments(g, seg);
    if (rc) return rc;
    const uint64_t n = seg[g->n];
    if (n == 0) return SF_OK;
    const uint32_t kb = g->key_bytes;
    if (kb == 4 && (reinterpret_cast<uintptr_t>(keys) & 3u))
        return fail(SF_EINVAL, "uint32 keys must be 4-byte aligned");
    if ((rc = check_gpu_ptr(keys, n * kb, "keys"))) return rc;
    if (kind == kMixed && (rc = check_gpu_ptr(ops, n, "ops"))) return rc;

    // Same plan as the previous call (same segments, buffers and op kind)?
    const uint32_t mode = kind == kMixed ? kOpsArray : kind == kDelete ? kAllDelete : kAllInsert;
    std::vector<TileDesc> old;
    old.swap(g->plan);
    build_plan(g, seg, static_cast<const uint8_t*>(keys), ops, mode);
    const bool same = g->plan_on_device && old.size() == g->plan.size() && g->plan_kind == kind &&
                      std::memcmp(old.data(), g->plan.data(), old.size() * sizeof(TileDesc)) == 0;
    const bool profiling = g->prof.on;
    if (!same) {
        drop_graph(g);
        hipError_t e = hipStreamSynchronize(g->stream);  // the old table may still be in use
        if (e != hipSuccess) return device_fail(e, "group sync");
        if ((rc = ensure_device_tiles(g->d_tiles, g->tiles_cap, g->plan.size()))) return rc;
        if ((rc = upload_tiles(g, g->d_tiles, g->plan))) return rc;
        if ((rc = upload_ranges(g))) return rc;
        g->plan_kind = kind;
        g->plan_on_device = true;
    }
    const bool ins = kind != kDelete, del = kind != kInsert;
    auto launch_all = [&](Profiler* prof) {
        if (kb == 4) launch_plan<4>(g, ins, del, prof);
        else launch_plan<13>(g, ins, del, prof);
    };
    if (!g->use_graph || profiling) {
        launch_all(profiling ? &g->prof : nullptr);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? SF_OK : device_fail(e, "group update launch");
    }
    if (!g->exec) {
        hipError_t e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return device_fail(e, "graph capture begin");
        launch_all(nullptr);
        e = hipStreamEndCapture(g->stream, &g->graph);
        if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            drop_graph(g);
            return device_fail(e, "graph capture");
        }
    }
    hipError_t e = hipGraphLaunch(g->exec, g->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "graph launch");
}

template <int KB, typename S>
void launch_group_query(sf_group* g, unsigned tiles) {
    const ListPlan<KB> plan{g->d_qtiles, g->d_desc};
    launch_query_rows<KB, ListPlan<KB>, S>(g->d_uniform, plan, tiles, g->stream);
}

}  // namespace

extern "C" {

uint64_t sf_group_footprint(uint32_t n, const sf_config* cfgs, uint64_t round_ops) {
    Layout L;
    if (layout_of(n, cfgs, round_ops, L)) return 0;
    return L.total;
}

int sf_group_create(uint32_t n, const sf_config* cfgs, uint64_t round_ops, uint64_t hbm_budget_bytes,
                    void* hip_stream, sf_group** out) {
    if (!out) return fail(SF_EINVAL, "null output handle");
    Layout L;
    int rc = layout_of(n, cfgs, round_ops, L);
    if (rc) return rc;
    if (hbm_budget_bytes && L.total > hbm_budget_bytes)
        return fail(SF_ENOMEM, "group needs " + std::to_string(L.total) + " bytes, budget is " +
                                   std::to_string(hbm_budget_bytes));
    sf_group* g = new sf_group{};
    g->n = n;
    g->key_bytes = cfgs[0].key_bytes;
    g->d_max = L.d_max;
    g->d_uniform = cfgs[0].d;
    for (uint32_t i = 1; i < n; i++)
        if (cfgs[i].d != cfgs[0].d) g->d_uniform = 0;
    g->cfg.assign(cfgs, cfgs + n);
    g->stream = static_cast<hipStream_t>(hip_stream);
    if (!g->stream) {
        hipError_t se = hipStreamCreate(&g->stream);  // default priority, blocking w.r.t. the null stream
        if (se != hipSuccess) {
            (void)hipGetLastError();
            delete g;
            return device_fail(se, "sf_group_create stream");
        }
        g->own_stream = true;
    }
    g->round_ops = L.round_ops;
    g->merge_round = L.merge_round;
    g->tile_j = 8;
    g->use_graph = true;
    g->merge = true;
    g->state_bytes = L.state;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&g->base), L.total - (L.owner ? L.owner_bytes() : 0));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (g->own_stream) (void)hipStreamDestroy(g->stream);
        delete g;
        return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "hipMalloc: out of device memory")
                                        : device_fail(e, "sf_group_create");
    }
    g->desc.resize(n);
    for (uint32_t i = 0; i < n; i++) {
        g->desc[i].g = geom_of(&cfgs[i]);
        g->desc[i].fat = reinterpret_cast<uint32_t*>(g->base + L.fat_off[i]);
        g->desc[i].slim = g->desc[i].fat + cfgs[i].z;
    }
    g->d_desc = reinterpret_cast<SketchDesc*>(g->base + L.desc);
    g->stage = reinterpret_cast<uint16_t*>(g->base + L.stage);
    g->bpre = reinterpret_cast<uint32_t*>(g->base + L.bpre);
    g->asnap = reinterpret_cast<uint16_t*>(g->base + L.asnap);
    g->part = g->base + L.part;
    g->ent_key = g->base + L.ent_key;
    g->ent_cnt = reinterpret_cast<uint32_t*>(g->base + L.ent_cnt);
    g->meta = reinterpret_cast<MergeMeta*>(g->base + L.meta);
    g->hist = reinterpret_cast<uint32_t*>(g->base + L.hist);
    g->chunks = reinterpret_cast<MergeChunk*>(g->base + L.chunks);
    g->hist_groups = part_groups_max(L.merge_round, kHistExtra);
    if (L.owner) {
        g->own_og = L.og;
        g->own_sizes[0] = L.pairs;
        g->own_sizes[1] = L.pos;
        g->own_sizes[2] = L.res;
        g->own_sizes[3] = L.level;
        g->own_sizes[4] = L.hmat;
        g->own_sizes[5] = L.pmeta;
        g->owner_ok = true;
        if ((rc = group_owner_alloc(g))) {
            (void)hipFree(g->base);
            if (g->own_stream) (void)hipStreamDestroy(g->stream);
            delete g;
            return rc;
        }
    }
    e = hipMemcpy(g->d_desc, g->desc.data(), n * sizeof(SketchDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(g->base, 0, L.state, g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g->meta, 0, sizeof(MergeMeta), g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        (void)hipFree(g->base);
        if (g->own_base) (void)hipFree(g->own_base);
        if (g->own_stream) (void)hipStreamDestroy(g->stream);
        delete g;
        return device_fail(e, "sf_group_create init");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(g);
    }
    *out = g;
    return SF_OK;
}

int sf_group_destroy(sf_group* g) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g || !g_live.erase(g)) return fail(SF_ESTATE, "group handle is not live");
    }
    hipError_t e = hipStreamSynchronize(g->stream);
    drop_graph(g);
    if (g->d_tiles) (void)hipFree(g->d_tiles);
    if (g->d_qtiles) (void)hipFree(g->d_qtiles);
    if (g->h_tiles) (void)hipHostFree(g->h_tiles);
    if (g->d_ranges) (void)hipFree(g->d_ranges);
    if (g->own_base) (void)hipFree(g->own_base);
    hipError_t e2 = hipFree(g->base);
    if (g->own_stream) (void)hipStreamDestroy(g->stream);
    delete g;
    if (e != hipSuccess) return device_fail(e, "sf_group_destroy sync");
    if (e2 != hipSuccess) return device_fail(e2, "sf_group_destroy free");
    return SF_OK;
}

int sf_group_reset(sf_group* g) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    hipError_t e = hipMemsetAsync(g->base, 0, g->state_bytes, g->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_group_reset");
}

int sf_group_insert(sf_group* g, const void* keys, const uint64_t* seg) {
    return group_updates(g, keys, nullptr, seg, kInsert);
}

int sf_group_delete(sf_group* g, const void* keys, const uint64_t* seg) {
    return group_updates(g, keys, nullptr, seg, kDelete);
}

int sf_group_update(sf_group* g, const void* keys, const uint8_t* ops, const uint64_t* seg) {
    return group_updates(g, keys, ops, seg, kMixed);
}

int sf_group_query(sf_group* g, const void* keys, const uint64_t* seg, uint32_t* out) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    int rc = check_segments(g, seg);
    if (rc) return rc;
    const uint64_t n = seg[g->n];
    if (n == 0) return SF_OK;
    const uint32_t kb = g->key_bytes;
    if (kb == 4 && (reinterpret_cast<uintptr_t>(keys) & 3u))
        return fail(SF_EINVAL, "uint32 keys must be 4-byte aligned");
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(SF_EINVAL, "out must be 4-byte aligned");
    if ((rc = check_gpu_ptr(keys, n * kb, "keys"))) return rc;
    if ((rc = check_gpu_ptr(out, n * 4, "out"))) return rc;
    // The same keys, answers and segments as the last call: its table is still
    // on the device (no upload, no wait).
    const bool same = g->q_keys == keys && g->q_out == out && g->q_seg.size() == size_t(g->n) + 1 &&
                      std::memcmp(g->q_seg.data(), seg, (size_t(g->n) + 1) * sizeof(uint64_t)) == 0;
    if (!same) {
        std::vector<TileDesc> tiles;
        const uint8_t* k8 = static_cast<const uint8_t*>(keys);
        for (uint32_t s = 0; s < g->n; s++)
            for (uint64_t lo = seg[s]; lo < seg[s + 1]; lo += kBlock) {
                TileDesc t{};
                t.keys = k8 + lo * kb;
                t.out = out + lo;
                t.count = uint32_t(std::min<uint64_t>(kBlock, seg[s + 1] - lo));
                t.sketch = s;
                t.mode = kAllInsert;
                tiles.push_back(t);
            }
        // Workgroup b runs on XCD b % 8: deal the tiles so that XCD x takes the
        // x-th eighth of them (whole runs of sketches), and a sketch's records
        // are cached in one L2 instead of eight.  Empty tiles pad the last turn.
        const size_t nt = tiles.size(), per = (nt + kXcds - 1) / kXcds;
        std::vector<TileDesc> dealt(per * kXcds, TileDesc{});
        for (size_t i = 0; i < nt; i++) {
            const size_t x = i / per, j = i % per;
            dealt[j * kXcds + x] = tiles[i];
        }
        hipError_t e = hipStreamSynchronize(g->stream);  // previous query table may be in use
        if (e != hipSuccess) return device_fail(e, "group sync");
        g->q_keys = nullptr;
        if ((rc = ensure_device_tiles(g->d_qtiles, g->qtiles_cap, dealt.size()))) return rc;
        if ((rc = upload_tiles(g, g->d_qtiles, dealt))) return rc;
        g->q_keys = keys;
        g->q_out = out;
        g->q_seg.assign(seg, seg + g->n + 1);
        g->q_tiles = dealt.size();
    }
    {
        Timed tm(&g->prof, g->stream, SF_K_QUERY, n);
        if (kb == 4) launch_group_query<4, uint32_t>(g, unsigned(g->q_tiles));
        else launch_group_query<13, uint32_t>(g, unsigned(g->q_tiles));
    }
    hipError_t e;
    e = hipGetLastError();
    return e == hipSuccess ? SF_OK : device_fail(e, "group query launch");
}

int sf_group_export_slim(sf_group* g, uint32_t i, uint16_t* out, uint64_t out_elems) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    if (i >= g->n) return fail(SF_EINVAL, "sketch index out of range");
    const uint64_t cells = uint64_t(g->cfg[i].d) * g->cfg[i].w;
    if (!out) return fail(SF_EINVAL, "out is null");
    if (out_elems < cells) return fail(SF_EINVAL, "out_elems < d*w");
    const bool host = host_dest(out);
    if (!host) {
        int rc = check_gpu_ptr(out, cells * 2, "out");
        if (rc) return rc;
    }
    uint16_t* dst = host ? g->stage : out;
    const unsigned grid = blocks_for(cells, kBlock) < 4096u ? blocks_for(cells, kBlock) : 4096u;
    k_pack16<uint32_t><<<dim3(grid), dim3(kBlock), 0, g->stream>>>(g->desc[i].slim, dst, cells, g->desc[i].g.rs, nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && host) e = hipMemcpyAsync(out, g->stage, cells * 2, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_group_export_slim");
}

int sf_group_export_fat(sf_group* g, uint32_t i, uint32_t* out, uint64_t out_elems) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    if (i >= g->n) return fail(SF_EINVAL, "sketch index out of range");
    const uint64_t n = uint64_t(g->cfg[i].d) * g->cfg[i].w * g->cfg[i].z;
    if (!out) return fail(SF_EINVAL, "out is null");
    if (out_elems < n) return fail(SF_EINVAL, "out_elems < d*w*z");
    const bool host = host_dest(out);
    if (!host) {
        int rc = check_gpu_ptr(out, n * 4, "out");
        if (rc) return rc;
    }
    uint32_t* dst = host ? reinterpret_cast<uint32_t*>(g->stage) : out;
    const unsigned grid = blocks_for(n, kBlock) < 4096u ? blocks_for(n, kBlock) : 4096u;
    k_unpack_fat<uint32_t><<<dim3(grid), dim3(kBlock), 0, g->stream>>>(
        g->desc[i].fat, dst, uint64_t(g->cfg[i].d) * g->cfg[i].w, g->cfg[i].z);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && host) e = hipMemcpyAsync(out, dst, n * 4, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_group_export_fat");
}

int sf_group_sync(sf_group* g) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    hipError_t e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_group_sync");
}

int sf_group_set_graph(sf_group* g, int enable) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    g->use_graph = enable != 0;
    return SF_OK;
}

int sf_group_set_tile(sf_group* g, uint32_t tile_ops) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    if (tile_ops != 256 && tile_ops != 1024 && tile_ops != 2048)
        return fail(SF_EINVAL, "tile_ops must be 256, 1024 or 2048");
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return device_fail(e, "group sync");
    g->tile_j = tile_ops / kBlock;
    drop_graph(g);
    g->plan_on_device = false;
    return SF_OK;
}

int sf_group_set_merge(sf_group* g, int mode) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    if (mode < 0 || mode > 2) return fail(SF_EINVAL, "group merge mode must be 0, 1 or 2");
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return device_fail(e, "group sync");
    int rc = SF_OK;
    if (mode == 1 && g->owner_ok && !g->own_base) rc = group_owner_alloc(g);
    if (mode != 1 && g->own_base) {
        (void)hipFree(g->own_base);
        g->own_base = nullptr;
    }
    g->merge = mode != 0;
    g->owner_on = mode == 1 && g->own_base;
    drop_graph(g);
    g->plan_on_device = false;
    return rc;
}

int sf_group_set_owner_ratio(sf_group* g, double ratio) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    if (!(ratio >= 0.0 && ratio <= 1e6)) return fail(SF_EINVAL, "owner ratio must be in [0, 1e6]");
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return device_fail(e, "group sync");
    g->own_ratio = ratio;
    drop_graph(g);
    g->plan_on_device = false;
    return SF_OK;
}

int sf_group_merge_path(sf_group* g) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    return !g->merge ? 0 : g->owner_on ? 1 : 2;
}

int sf_group_merge_stats(sf_group* g, uint64_t* insert_entries, uint64_t* delete_entries) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    unsigned long long acc[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(acc, &g->meta->acc_ins, sizeof(acc), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return device_fail(e, "sf_group_merge_stats");
    if (insert_entries) *insert_entries = acc[0];
    if (delete_entries) *delete_entries = acc[1];
    return SF_OK;
}

int sf_group_rounds(sf_group* g, uint64_t* subrounds, uint64_t* tiles) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    if (subrounds) *subrounds = g->subrounds.size();
    if (tiles) *tiles = g->plan.size();
    return SF_OK;
}

int sf_group_profile(sf_group* g, int enable) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    g->prof.on = enable != 0;
    return SF_OK;
}

int sf_group_profile_read(sf_group* g, sf_kernel_stats* out, int reset) {
    if (!live(g)) return fail(SF_ESTATE, "group handle is not live");
    int rc = g->prof.drain();
    if (out) *out = g->prof.acc;
    if (reset) g->prof.acc = sf_kernel_stats{};
    return rc;
}

}  // extern "C"
