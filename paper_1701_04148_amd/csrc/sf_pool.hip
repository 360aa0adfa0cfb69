// libsf.so: sketch pools -- the device side of a serving loop.
//
// A pool holds `slots` sketches of one shape in one allocation sized by an
// HBM budget.  Streams (monitoring nodes) acquire a slot when admitted and
// release it when they close.  sf_pool_launch takes requests of many slots
// at once -- at most one per slot -- and runs them with shared launches:
// every update request is cut into its own schedule batches (each request
// starts a new batch, exactly as one sf_insert / sf_delete / sf_update call on
// a lone sketch would), round k runs batch k of every update request, and
// the query requests run in one query launch.  A slot's result is therefore
// the same alone and in any mix.  Launches are queued on the pool's stream
// and complete in order; each returns a ticket backed by a HIP event.
//
// Update sub-rounds take the batch-merge path by default (duplicate (key,
// slot) pairs merged across the sub-round, S1..S5 once per merged entry);
// merged sub-rounds hold at most 2^24 ops, or one batch if larger.  For slots
// of at most 64 MiB of records, a request batch of at least owner_ratio * w
// ops takes owner-computes S1..S5 (its slot's (row, range) tiles staged in
// LDS) and the others the atomic entry kernels, in the same sub-round; a
// sub-round's owner batches hold at most 2^22 ops, and its range table
// travels in the descriptor ring beside its tiles.
//
// Tile descriptors of in-flight launches live in a device ring; a region is
// reused only after the launch that reads it has completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "sf.h"
#include "sf_host.hpp"

using namespace sfk;
using namespace sfh;

struct sf_pool {
    sf_config cfg;
    uint32_t slots;
    uint64_t slot_bytes;           // one slot's cell records (Fat bucket + Slim per cell), rounded
    hipStream_t stream;
    bool own_stream;
    char* base;
    SketchDesc* d_desc;
    std::vector<SketchDesc> desc;
    uint32_t* bpre;
    uint16_t* asnap;
    uint16_t* stage;
    uint64_t round_ops;
    uint64_t merge_round;          // ops of a merged sub-round
    void* part;                    // merge buffers, merge_round entries each
    void* ent_key;
    uint32_t* ent_cnt;
    MergeMeta* meta;
    uint32_t* hist;                // per-group bucket histograms of a merged sub-round
    MergeChunk* chunks;            // key range of every merge chunk of a merged sub-round
    uint64_t hist_groups;          // partition groups (tiles) a merged sub-round may have
    uint32_t tile_j;
    bool merge;
    std::vector<uint8_t> in_use;
    std::vector<uint32_t> free_list;
    TileDesc* d_ring;
    size_t ring_cap;
    size_t ring_head;
    struct Flight {
        uint64_t ticket;
        size_t begin, end;
        hipEvent_t ev;
        std::vector<TileDesc> host;  // source of the tile upload, kept until done
    };
    std::deque<Flight> flights;
    uint64_t next_ticket;
    uint64_t done_upto;  // every ticket <= done_upto has completed
    std::vector<hipEvent_t> spare;
    Profiler prof;
    // owner-computes S1..S5 (slots whose records are small enough to stream)
    bool owner_ok = false;
    double own_ratio = 0.5;        // a batch is owner-computed when its ops >= own_ratio * w
    uint64_t owner_ops = 0;        // owner batches' ops per sub-round at most
    OwnerGeom own_og{};
    OwnerBufs own{};
};

namespace {

std::mutex g_mu;
std::unordered_set<const sf_pool*> g_live;

bool live(const sf_pool* p) {
    std::lock_guard<std::mutex> lk(g_mu);
    return p && g_live.count(p);
}

constexpr size_t kRingTiles = size_t(1) << 21;  // 2M tiles (80 MiB) of in-flight descriptors
constexpr uint64_t kHistExtra = 1024;            // partial tiles (one per request) a merged sub-round may add

struct PoolLayout {
    uint64_t slot_bytes, per_slot, shared, round_ops, merge_round, mkey;
    bool owner = false;
    OwnerGeom og{};
    uint64_t owner_ops = 0, pairs = 0, pos = 0, res = 0, level = 0, hmat = 0, pmeta = 0;
};

struct SubRound {
    uint32_t first, tiles;
    uint64_t ops;
    uint32_t ranges = 0;           // owner path: ranges per row of its owner batches
    bool atomic_side = false;      // ... beside batches on the atomic entry kernels
    uint64_t table = 0;            // ... offset of its range table (words) in the launch's table area
};

constexpr uint64_t kPoolOwnerSlotBytes = 64ull << 20;  // slots whose records the owner path may stream
constexpr uint64_t kPoolOwnerOps = 1ull << 22;         // owner batches' ops per sub-round

// Owner layout of a pool's slots: one slot's ranges as large as a range's Fat
// counters allow, all of them within one sub-round's range table.
bool pool_owner_geom(const sf_config* c, OwnerGeom* og) {
    if (uint64_t(c->d) * c->w * (c->z + 1) * 4 > kPoolOwnerSlotBytes) return false;
    uint32_t zbits = 0;
    while ((1ull << zbits) < c->z) zbits++;
    uint32_t sh = 4;
    while ((2ull << sh) * c->z <= kOwnCounters && ((2ull << sh) << zbits) <= 65536) sh++;
    if ((1ull << sh) * c->z > kOwnCounters || ((1ull << sh) << zbits) > 65536) return false;
    const uint32_t qcap = std::min<uint32_t>(kMaxRanges, kMaxCols / (2 * c->d));
    if (((uint64_t(c->w) + (1ull << sh) - 1) >> sh) > qcap) return false;
    *og = OwnerGeom{};
    og->cr_shift = sh;
    og->zbits = zbits;
    og->d = c->d;
    return true;
}

PoolLayout pool_layout(const sf_config* c, uint64_t round_ops) {
    PoolLayout L;
    const uint64_t cells = uint64_t(c->d) * c->w;
    L.slot_bytes = round256(cells * (c->z + 1) * 4);
    L.per_slot = L.slot_bytes + round256(sizeof(SketchDesc));
    L.round_ops = std::max<uint64_t>(round_ops ? round_ops : (1ull << 24), c->batch_ops);
    L.merge_round = std::max<uint64_t>(std::min<uint64_t>(L.round_ops, 1ull << 24), c->batch_ops);
    L.mkey = c->key_bytes == 4 ? sizeof(MKey<4, true>) : sizeof(MKey<13, true>);
    L.shared = round256(uint64_t(c->d) * L.round_ops * 4) + round256(uint64_t(c->d) * L.round_ops * 2) +
               round256(cells * c->z * 4) + round256(kRingTiles * sizeof(TileDesc)) +
               2 * round256(L.merge_round * L.mkey) + round256(L.merge_round * 4) + round256(sizeof(MergeMeta)) +
               round256(part_groups_max(L.merge_round, kHistExtra) * 2 * kMaxBuckets * 4) +
               round256(merge_chunks_max(L.merge_round) * sizeof(MergeChunk));
    L.owner = pool_owner_geom(c, &L.og);
    if (L.owner) {
        // pairs and their snapshots for the owner batches; positions and T
        // for every entry of a sub-round; column counts for all its tiles
        const uint64_t d = c->d, mr = L.merge_round;
        const uint32_t qcap = std::min<uint32_t>(kMaxRanges, kMaxCols / (2 * c->d));
        L.owner_ops = std::min(mr, kPoolOwnerOps);
        L.pairs = round256(d * L.owner_ops * 8);
        L.pos = round256(d * mr * 4);
        L.res = round256(d * L.owner_ops * 8);
        L.level = round256(mr * 2);
        L.hmat = round256(uint64_t(pair_tiles_max(uint32_t(mr))) * 2 * d * qcap * 4);
        L.pmeta = round256(sizeof(PairMeta));
        L.shared += L.pairs + L.pos + L.res + L.level + L.hmat + L.pmeta;
    }
    return L;
}

int retire(sf_pool* p, bool block_oldest) {
    while (!p->flights.empty()) {
        auto& f = p->flights.front();
        hipError_t e = block_oldest ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();
            return SF_OK;
        }
        if (e != hipSuccess) return device_fail(e, "pool launch");
        p->done_upto = f.ticket;
        p->spare.push_back(f.ev);
        p->flights.pop_front();
        block_oldest = false;
    }
    return SF_OK;
}

// A contiguous region of k ring entries that no in-flight launch reads.
int ring_alloc(sf_pool* p, size_t k, size_t* begin) {
    if (k > p->ring_cap) return fail(SF_EINVAL, "launch has more tiles than the descriptor ring holds");
    for (;;) {
        if (p->flights.empty()) p->ring_head = 0;
        size_t b = p->ring_head + k <= p->ring_cap ? p->ring_head : 0;
        bool clash = false;
        for (auto& f : p->flights)
            if (b < f.end && f.begin < b + k) clash = true;
        if (!clash) {
            *begin = b;
            p->ring_head = b + k;
            return SF_OK;
        }
        int rc = retire(p, true);
        if (rc) return rc;
    }
}

template <int KB>
void launch_updates(sf_pool* p, const TileDesc* d_tiles, const std::vector<SubRound>& subs,
                    const std::vector<TileDesc>& host, const uint32_t* d_tables) {
    MergeRun<KB, true> run{static_cast<MKey<KB, true>*>(p->part), static_cast<MKey<KB, true>*>(p->ent_key),
                           p->ent_cnt, p->meta, p->hist, p->chunks, uint32_t(p->merge_round), p->bpre,
                           p->asnap,
                           uint32_t(p->round_ops)};
    const SketchTable table{p->d_desc};
    for (auto& sr : subs) {
        bool ins = false, del = false;
        for (uint32_t t = 0; t < sr.tiles; t++) {
            const TileDesc& td = host[sr.first + t];
            ins = ins || td.mode != kAllDelete;
            del = del || td.mode != kAllInsert;
        }
        const ListPlan<KB> plan{d_tiles + sr.first, p->d_desc};
        const uint32_t cnt = uint32_t(sr.ops);
        run.own = nullptr;
        if (p->merge && sr.ranges) {  // owner-computed batches in this sub-round
            const uint32_t* tab = d_tables + sr.table;
            run.own = &p->own;
            run.side_atomic = sr.atomic_side;
            run.sub_og = p->own_og;
            run.sub_og.R = sr.ranges;
            run.sub_og.ncol = 2 * p->own_og.d * sr.ranges;
            run.sub_og.xcd = (kXcds % p->own_og.d == 0 && (p->own_og.d * sr.ranges) % kXcds == 0) ? 1u : 0u;
            run.sub_rm = TableRanges{tab, tab + p->slots, tab + p->slots + sr.ranges};
            run.max_z = p->cfg.z;
        }
        if (!p->merge) {
            Steps<ListPlan>::by_rows<KB>(p->cfg.d, p->tile_j, plan, sr.tiles, ins, del, p->bpre, p->asnap,
                                        uint32_t(p->round_ops), p->stream, &p->prof, cnt);
        } else if (p->cfg.d == 4) {
            run.template launch<4>(plan, sr.tiles, cnt, table, ins, del, p->stream, &p->prof);
        } else if (p->cfg.d == 8) {
            run.template launch<8>(plan, sr.tiles, cnt, table, ins, del, p->stream, &p->prof);
        } else {
            run.template launch<0>(plan, sr.tiles, cnt, table, ins, del, p->stream, &p->prof);
        }
    }
}

}  // namespace

extern "C" {

uint64_t sf_pool_slot_bytes(const sf_config* cfg) {
    if (validate(cfg)) return 0;
    return pool_layout(cfg, 0).per_slot;
}

int sf_pool_create(const sf_config* cfg, uint32_t max_slots, uint64_t round_ops, uint64_t hbm_budget_bytes,
                   void* hip_stream, sf_pool** out) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!out) return fail(SF_EINVAL, "null output handle");
    const PoolLayout L = pool_layout(cfg, round_ops);
    if (L.round_ops > (1ull << 31)) return fail(SF_EINVAL, "round_ops must be <= 2^31");
    uint64_t slots = max_slots;
    if (hbm_budget_bytes) {
        if (hbm_budget_bytes < L.shared + L.per_slot)
            return fail(SF_ENOMEM, "budget holds no slot (shared " + std::to_string(L.shared) + " + slot " +
                                       std::to_string(L.per_slot) + " bytes)");
        slots = std::min<uint64_t>(slots ? slots : ~0ull, (hbm_budget_bytes - L.shared) / L.per_slot);
    }
    if (slots == 0 || slots > (1u << 24)) return fail(SF_EINVAL, "slots must be in 1..2^24");
    sf_pool* p = new sf_pool{};
    p->cfg = *cfg;
    p->slots = uint32_t(slots);
    p->slot_bytes = L.slot_bytes;
    p->round_ops = L.round_ops;
    p->merge_round = L.merge_round;
    p->tile_j = 8;
    p->merge = true;
    p->ring_cap = kRingTiles;
    p->next_ticket = 1;
    p->stream = static_cast<hipStream_t>(hip_stream);
    if (!p->stream) {
        hipError_t se = hipStreamCreate(&p->stream);
        if (se != hipSuccess) {
            (void)hipGetLastError();
            delete p;
            return device_fail(se, "sf_pool_create stream");
        }
        p->own_stream = true;
    }
    const uint64_t state = slots * L.slot_bytes;
    const uint64_t total = state + round256(slots * sizeof(SketchDesc)) + L.shared;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->base), total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (p->own_stream) (void)hipStreamDestroy(p->stream);
        delete p;
        return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "hipMalloc: out of device memory")
                                        : device_fail(e, "sf_pool_create");
    }
    char* q = p->base + state;
    p->d_desc = reinterpret_cast<SketchDesc*>(q);
    q += round256(slots * sizeof(SketchDesc));
    p->bpre = reinterpret_cast<uint32_t*>(q);
    q += round256(uint64_t(cfg->d) * L.round_ops * 4);
    p->asnap = reinterpret_cast<uint16_t*>(q);
    q += round256(uint64_t(cfg->d) * L.round_ops * 2);
    p->stage = reinterpret_cast<uint16_t*>(q);
    q += round256(uint64_t(cfg->d) * cfg->w * cfg->z * 4);
    p->d_ring = reinterpret_cast<TileDesc*>(q);
    q += round256(kRingTiles * sizeof(TileDesc));
    p->part = q;
    q += round256(L.merge_round * L.mkey);
    p->ent_key = q;
    q += round256(L.merge_round * L.mkey);
    p->ent_cnt = reinterpret_cast<uint32_t*>(q);
    q += round256(L.merge_round * 4);
    p->meta = reinterpret_cast<MergeMeta*>(q);
    q += round256(sizeof(MergeMeta));
    p->hist = reinterpret_cast<uint32_t*>(q);
    p->hist_groups = part_groups_max(L.merge_round, kHistExtra);
    q += round256(p->hist_groups * 2 * kMaxBuckets * 4);
    p->chunks = reinterpret_cast<MergeChunk*>(q);
    q += round256(merge_chunks_max(L.merge_round) * sizeof(MergeChunk));
    if (L.owner) {
        p->owner_ok = true;
        p->owner_ops = L.owner_ops;
        p->own_og = L.og;
        p->own.og = L.og;
        p->own.pairs[0] = reinterpret_cast<uint64_t*>(q);
        q += L.pairs;
        p->own.pos = reinterpret_cast<uint32_t*>(q);
        q += L.pos;
        p->own.res = reinterpret_cast<uint64_t*>(q);
        q += L.res;
        p->own.level = reinterpret_cast<uint16_t*>(q);
        q += L.level;
        p->own.hmat = reinterpret_cast<uint32_t*>(q);
        q += L.hmat;
        p->own.pm[0] = reinterpret_cast<PairMeta*>(q);
        q += L.pmeta;
    }
    p->desc.resize(slots);
    const Geom geo = geom_of(cfg);
    for (uint64_t i = 0; i < slots; i++) {
        p->desc[i].g = geo;
        p->desc[i].fat = reinterpret_cast<uint32_t*>(p->base + i * L.slot_bytes);
        p->desc[i].slim = p->desc[i].fat + cfg->z;
    }
    e = hipMemcpy(p->d_desc, p->desc.data(), slots * sizeof(SketchDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(p->meta, 0, sizeof(MergeMeta), p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        (void)hipFree(p->base);
        if (p->own_stream) (void)hipStreamDestroy(p->stream);
        delete p;
        return device_fail(e, "sf_pool_create table");
    }
    p->in_use.assign(slots, 0);
    for (uint64_t i = slots; i-- > 0;) p->free_list.push_back(uint32_t(i));
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(p);
    }
    *out = p;
    return SF_OK;
}

int sf_pool_destroy(sf_pool* p) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!p || !g_live.erase(p)) return fail(SF_ESTATE, "pool handle is not live");
    }
    hipError_t e = hipStreamSynchronize(p->stream);
    for (auto& f : p->flights) (void)hipEventDestroy(f.ev);
    for (auto ev : p->spare) (void)hipEventDestroy(ev);
    hipError_t e2 = hipFree(p->base);
    if (p->own_stream) (void)hipStreamDestroy(p->stream);
    delete p;
    if (e != hipSuccess) return device_fail(e, "sf_pool_destroy sync");
    if (e2 != hipSuccess) return device_fail(e2, "sf_pool_destroy free");
    return SF_OK;
}

int sf_pool_capacity(sf_pool* p, uint32_t* slots, uint32_t* free_slots) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    if (slots) *slots = p->slots;
    if (free_slots) *free_slots = uint32_t(p->free_list.size());
    return SF_OK;
}

int sf_pool_acquire(sf_pool* p, uint32_t* slot) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    if (!slot) return fail(SF_EINVAL, "null slot pointer");
    if (p->free_list.empty()) return fail(SF_ENOMEM, "no free slot in the pool's HBM budget");
    const uint32_t s = p->free_list.back();
    // zeroed on the pool stream: ordered after every launch that used the slot before
    hipError_t e = hipMemsetAsync(p->desc[s].fat, 0, p->slot_bytes, p->stream);
    if (e != hipSuccess) return device_fail(e, "sf_pool_acquire");
    p->free_list.pop_back();
    p->in_use[s] = 1;
    *slot = s;
    return SF_OK;
}

int sf_pool_release(sf_pool* p, uint32_t slot) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    if (slot >= p->slots || !p->in_use[slot]) return fail(SF_EINVAL, "slot is not acquired");
    p->in_use[slot] = 0;
    p->free_list.push_back(slot);
    return SF_OK;
}

int sf_pool_launch(sf_pool* p, const sf_request* reqs, uint32_t n, uint64_t* ticket) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    if (n && !reqs) return fail(SF_EINVAL, "null request array");
    int rc = retire(p, false);
    if (rc) return rc;
    const uint32_t kb = p->cfg.key_bytes;
    std::vector<uint8_t> seen(p->slots, 0);
    for (uint32_t r = 0; r < n; r++) {
        const sf_request& q = reqs[r];
        if (q.slot >= p->slots || !p->in_use[q.slot]) return fail(SF_EINVAL, "request for a slot that is not acquired");
        if (seen[q.slot]) return fail(SF_EINVAL, "at most one request per slot per launch");
        seen[q.slot] = 1;
        if (q.kind > SF_REQ_QUERY) return fail(SF_EINVAL, "bad request kind");
        if (q.n == 0) continue;
        if (kb == 4 && (reinterpret_cast<uintptr_t>(q.keys) & 3u))
            return fail(SF_EINVAL, "uint32 keys must be 4-byte aligned");
        if ((rc = check_gpu_ptr(q.keys, q.n * kb, "keys"))) return rc;
        if (q.kind == SF_REQ_UPDATE && (rc = check_gpu_ptr(q.ops, q.n, "ops"))) return rc;
        if (q.kind == SF_REQ_QUERY) {
            if (reinterpret_cast<uintptr_t>(q.out) & 3u) return fail(SF_EINVAL, "out must be 4-byte aligned");
            if ((rc = check_gpu_ptr(q.out, q.n * 4, "out"))) return rc;
        }
    }
    // update tiles: round k = batch k of every update request; sub-rounds bounded by
    // round_ops (merged: merge_round, tiles of kPartOps ops for the partition kernels)
    const uint32_t tile_ops = p->merge ? kPartOps : uint32_t(kBlock) * p->tile_j;
    const uint64_t limit = p->merge ? p->merge_round : p->round_ops;
    const uint64_t max_tiles = p->merge ? p->hist_groups : ~0ull;
    const uint64_t b = p->cfg.batch_ops;
    // owner path: a batch of at least own_ratio * w ops (and at most the owner
    // buffers' share of a sub-round) streams its slot's ranges; a sub-round
    // holds at most qcap ranges per row of such batches
    const bool owner = p->merge && p->owner_ok;
    const uint32_t qcap = owner ? std::min<uint32_t>(kMaxRanges, kMaxCols / (2 * p->cfg.d)) : 0u;
    const uint32_t slot_ranges =
        owner ? uint32_t((uint64_t(p->cfg.w) + (1ull << p->own_og.cr_shift) - 1) >> p->own_og.cr_shift) : 0u;
    auto owns = [&](uint64_t cnt) {
        return owner && cnt <= p->owner_ops && double(cnt) >= p->own_ratio * double(p->cfg.w);
    };
    std::vector<TileDesc> tiles;
    std::vector<SubRound> subs;
    uint64_t rounds = 0;
    for (uint32_t r = 0; r < n; r++)
        if (reqs[r].kind != SF_REQ_QUERY) rounds = std::max(rounds, (reqs[r].n + b - 1) / b);
    for (uint64_t k = 0; k < rounds; k++) {
        uint64_t used = 0, own_used = 0;
        uint32_t first = uint32_t(tiles.size()), nq = 0;
        bool side = false;
        for (uint32_t r = 0; r < n; r++) {
            const sf_request& q = reqs[r];
            if (q.kind == SF_REQ_QUERY || k * b >= q.n) continue;
            const uint64_t lo = k * b, cnt = std::min(b, q.n - lo);
            const uint64_t ntiles = (cnt + tile_ops - 1) / tile_ops;
            const bool o = owns(cnt);
            if (used && (used + cnt > limit || tiles.size() - first + ntiles > max_tiles ||
                         (o && (nq + slot_ranges > qcap || own_used + cnt > p->owner_ops)))) {
                subs.push_back({first, uint32_t(tiles.size()) - first, used, nq, side});
                first = uint32_t(tiles.size());
                used = own_used = 0;
                nq = 0;
                side = false;
            }
            if (o) {
                nq += slot_ranges;
                own_used += cnt;
            } else {
                side = side || owner;
            }
            const uint32_t mode = q.kind == SF_REQ_UPDATE ? kOpsArray
                                  : q.kind == SF_REQ_DELETE ? kAllDelete : kAllInsert;
            for (uint64_t off = 0; off < cnt; off += tile_ops) {
                TileDesc t{};
                t.keys = static_cast<const uint8_t*>(q.keys) + (lo + off) * kb;
                t.ops = mode == kOpsArray ? q.ops + lo + off : nullptr;
                t.count = uint32_t(std::min<uint64_t>(tile_ops, cnt - off));
                t.sketch = q.slot;
                t.scr = uint32_t(used + off);
                t.mode = mode;
                tiles.push_back(t);
            }
            used += cnt;
        }
        if (uint32_t(tiles.size()) > first) subs.push_back({first, uint32_t(tiles.size()) - first, used, nq, side});
    }
    const size_t n_update_tiles = tiles.size();
    // range tables of the owner sub-rounds: per slot its first range (~0:
    // none), then per range its slot and its index in that slot
    std::vector<uint32_t> tab;
    for (auto& sr : subs) {
        if (!sr.ranges) continue;
        sr.table = tab.size();
        tab.resize(sr.table + p->slots + 2ull * sr.ranges, ~0u);
        uint32_t* qbase = tab.data() + sr.table;
        uint32_t* qsk = qbase + p->slots;
        uint32_t* qr = qsk + sr.ranges;
        uint32_t qn = 0;
        for (uint32_t t = sr.first; t < sr.first + sr.tiles;) {
            const uint32_t slot = tiles[t].sketch;
            uint64_t cnt = 0;  // the request's batch: its consecutive tiles
            for (; t < sr.first + sr.tiles && tiles[t].sketch == slot; t++) cnt += tiles[t].count;
            if (!owns(cnt)) continue;
            qbase[slot] = qn;
            for (uint32_t i = 0; i < slot_ranges; i++, qn++) {
                qsk[qn] = slot;
                qr[qn] = i;
            }
        }
    }
    for (uint32_t r = 0; r < n; r++) {
        const sf_request& q = reqs[r];
        if (q.kind != SF_REQ_QUERY) continue;
        for (uint64_t lo = 0; lo < q.n; lo += kBlock) {
            TileDesc t{};
            t.keys = static_cast<const uint8_t*>(q.keys) + lo * kb;
            t.out = q.out + lo;
            t.count = uint32_t(std::min<uint64_t>(kBlock, q.n - lo));
            t.sketch = q.slot;
            t.mode = kAllInsert;
            tiles.push_back(t);
        }
    }
    const size_t n_query_tiles = tiles.size() - n_update_tiles;
    // the tables ride in the descriptor ring after the tiles (same lifetime)
    const size_t tab_tiles = (tab.size() * 4 + sizeof(TileDesc) - 1) / sizeof(TileDesc);
    const size_t tab_first = tiles.size();
    tiles.resize(tiles.size() + tab_tiles, TileDesc{});
    if (tab_tiles) std::memcpy(tiles.data() + tab_first, tab.data(), tab.size() * 4);
    size_t begin = 0;
    if (!tiles.empty() && (rc = ring_alloc(p, tiles.size(), &begin))) return rc;
    sf_pool::Flight f;
    f.ticket = p->next_ticket;
    f.begin = begin;
    f.end = begin + tiles.size();
    f.host = std::move(tiles);
    hipError_t e = hipSuccess;
    if (!f.host.empty())
        e = hipMemcpyAsync(p->d_ring + begin, f.host.data(), f.host.size() * sizeof(TileDesc),
                           hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return device_fail(e, "tile upload");
    const uint32_t* d_tables = reinterpret_cast<const uint32_t*>(p->d_ring + begin + tab_first);
    if (kb == 4) launch_updates<4>(p, p->d_ring + begin, subs, f.host, d_tables);
    else launch_updates<13>(p, p->d_ring + begin, subs, f.host, d_tables);
    if (n_query_tiles) {
        uint64_t items = 0;
        for (size_t t = n_update_tiles; t < n_update_tiles + n_query_tiles; t++) items += f.host[t].count;
        Timed tm(&p->prof, p->stream, SF_K_QUERY, items);
        if (kb == 4) {
            const ListPlan<4> plan{p->d_ring + begin + n_update_tiles, p->d_desc};
            launch_query_rows<4, ListPlan<4>, uint32_t>(p->cfg.d, plan, unsigned(n_query_tiles), p->stream);
        } else {
            const ListPlan<13> plan{p->d_ring + begin + n_update_tiles, p->d_desc};
            launch_query_rows<13, ListPlan<13>, uint32_t>(p->cfg.d, plan, unsigned(n_query_tiles), p->stream);
        }
    }
    if ((e = hipGetLastError()) != hipSuccess) return device_fail(e, "pool launch");
    if (!p->spare.empty()) {
        f.ev = p->spare.back();
        p->spare.pop_back();
    } else if ((e = hipEventCreateWithFlags(&f.ev, hipEventDisableTiming)) != hipSuccess) {
        return device_fail(e, "pool event");
    }
    if ((e = hipEventRecord(f.ev, p->stream)) != hipSuccess) return device_fail(e, "pool event record");
    p->flights.push_back(std::move(f));
    if (ticket) *ticket = p->next_ticket;
    p->next_ticket++;
    return SF_OK;
}

int sf_pool_done(sf_pool* p, uint64_t ticket) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    int rc = retire(p, false);
    if (rc) return rc;
    return ticket <= p->done_upto ? 1 : 0;
}

int sf_pool_wait(sf_pool* p, uint64_t ticket) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    while (ticket > p->done_upto && !p->flights.empty()) {
        int rc = retire(p, true);
        if (rc) return rc;
    }
    return SF_OK;
}

int sf_pool_export_slim(sf_pool* p, uint32_t slot, uint16_t* out, uint64_t out_elems, int async) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    if (slot >= p->slots || !p->in_use[slot]) return fail(SF_EINVAL, "slot is not acquired");
    const uint64_t cells = uint64_t(p->cfg.d) * p->cfg.w;
    if (!out) return fail(SF_EINVAL, "out is null");
    if (out_elems < cells) return fail(SF_EINVAL, "out_elems < d*w");
    const bool host = host_dest(out);
    if (host && async) return fail(SF_EINVAL, "asynchronous export needs a device destination");
    if (!host) {
        int rc = check_gpu_ptr(out, cells * 2, "out");
        if (rc) return rc;
    }
    uint16_t* dst = host ? p->stage : out;
    const unsigned grid = blocks_for(cells, kBlock) < 4096u ? blocks_for(cells, kBlock) : 4096u;
    k_pack16<uint32_t><<<dim3(grid), dim3(kBlock), 0, p->stream>>>(p->desc[slot].slim, dst, cells, p->desc[slot].g.rs, nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && host) e = hipMemcpyAsync(out, p->stage, cells * 2, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess && !async) e = hipStreamSynchronize(p->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_pool_export_slim");
}

int sf_pool_export_fat(sf_pool* p, uint32_t slot, uint32_t* out, uint64_t out_elems) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    if (slot >= p->slots || !p->in_use[slot]) return fail(SF_EINVAL, "slot is not acquired");
    const uint64_t n = uint64_t(p->cfg.d) * p->cfg.w * p->cfg.z;
    if (!out) return fail(SF_EINVAL, "out is null");
    if (out_elems < n) return fail(SF_EINVAL, "out_elems < d*w*z");
    const bool host = host_dest(out);
    if (!host) {
        int rc = check_gpu_ptr(out, n * 4, "out");
        if (rc) return rc;
    }
    uint32_t* dst = host ? reinterpret_cast<uint32_t*>(p->stage) : out;
    const unsigned grid = blocks_for(n, kBlock) < 4096u ? blocks_for(n, kBlock) : 4096u;
    k_unpack_fat<uint32_t><<<dim3(grid), dim3(kBlock), 0, p->stream>>>(
        p->desc[slot].fat, dst, uint64_t(p->cfg.d) * p->cfg.w, p->cfg.z);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && host) e = hipMemcpyAsync(out, dst, n * 4, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_pool_export_fat");
}

int sf_pool_sync(sf_pool* p) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return device_fail(e, "sf_pool_sync");
    return retire(p, false);
}

int sf_pool_set_tile(sf_pool* p, uint32_t tile_ops) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    if (tile_ops != 256 && tile_ops != 1024 && tile_ops != 2048)
        return fail(SF_EINVAL, "tile_ops must be 256, 1024 or 2048");
    p->tile_j = tile_ops / kBlock;
    return SF_OK;
}

int sf_pool_set_merge(sf_pool* p, int batch_wide) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    p->merge = batch_wide != 0;
    return SF_OK;
}

int sf_pool_set_owner_ratio(sf_pool* p, double ratio) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    if (!p->owner_ok) return fail(SF_EINVAL, "this pool's slots do not take the owner-computes path");
    if (!(ratio >= 0.0 && ratio <= 1e6)) return fail(SF_EINVAL, "owner ratio must be in [0, 1e6]");
    p->own_ratio = ratio;
    return SF_OK;
}

int sf_pool_merge_stats(sf_pool* p, uint64_t* insert_entries, uint64_t* delete_entries) {
    if (!live(p)) return fail(SF_ESTATE, "pool handle is not live");
    unsigned long long acc[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(acc, &p->meta->acc_ins, sizeof(acc), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return device_fail(e, "sf_pool_merge_stats");
    if (insert_entries) *insert_entries = acc[0];
    if (delete_entries) *delete_entries = acc[1];
    return SF_OK;
}

}  // extern "C"
