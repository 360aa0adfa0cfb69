// libsf.so: SF-sketch hot path on MI355X (gfx950) behind the C ABI of sf.h,
// single-sketch entry points (sketch groups live in sf_group.hip).
//
// Device state of one sketch (all in HBM, one allocation made by sf_create):
//   rec   uint32 [d][w][z+1]  one record per cell: the cell's Fat bucket (z
//                             counters, Section 3.4) then the cell's Slim
//                             working copy, so S1, S3 and S5 read the Fat
//                             counter and the Slim counter of a cell from one
//                             cache line.  Slim values stay <= 65535 (the
//                             uint16 export is a narrowing copy); 32-bit cells
//                             give native atomic max / min.  fat points at
//                             the records, slim at word z of the first one.
//   stage                     export staging for host destinations (the larger
//                             of the dense uint16 Slim and uint32 Fat)
//   bpre  uint32 [d][b]     per-batch snapshot of insert ops' Fat counters
//   asnap uint16 [d][b]     per-batch snapshot of their Slim counters
// Each schedule batch runs the five steps of sf_kernels.hpp on the sketch's
// stream, over tiles of 256 * tile_j consecutive ops (UniformPlan).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "sf.h"
#include "sf_host.hpp"

using namespace sfk;
using namespace sfh;

namespace sfh {
std::string& last_error() {
    static thread_local std::string err;
    return err;
}
}  // namespace sfh

constexpr uint32_t kMaxQueryStreams = 16;

struct sf_sketch {
    sf_config cfg;
    Geom g;
    hipStream_t stream;
    int device;
    uint32_t* fat;
    uint32_t* slim;
    uint16_t* stage;
    uint64_t stage_bytes;  // also the per-row query scratch (stream-ordered like the exports)
    uint16_t* view;   // dense uint16 Slim as of the last export (queries read it while fresh)
    bool view_fresh;  // no update or reset since view was packed
    uint32_t* bpre;
    uint16_t* asnap;
    uint32_t stride;  // snapshot capacity in ops (= batch_ops)
    uint32_t tile_j;  // ops per thread of a tile (tile = 256 * tile_j ops)
    bool merge_batch; // merge duplicates across the whole batch (else per tile)
    void* part;       // batch merge: keys partitioned by bucket      [b] keys
    void* ent_key;    // batch merge: one key per merged entry        [b] keys
    uint32_t* ent_cnt;//              its op count                    [b]
    uint32_t* hist;   //              per-group bucket histograms     [b/8192+1][2048]
    MergeChunk* chunks;//             key range of every merge chunk
    MergeMeta* meta;
    bool owner_ok;    // the shape fits the owner-computes path
    bool owner_on;    // S1..S5 by (row, cell range) owners for large batches (else the entry kernels)
    bool owner_all;   // ... for every batch, however small (merge mode 3)
    int streams = -1; // owner path: partition side on a second stream (1), not (0), by batch size (-1)
    OwnerBufs own;
    char* own_base = nullptr;  // the owner path's buffers: their own allocation, held while mode 1 is set
    Profiler prof;
    // host-fed updates (sf_update_host): two device chunk buffers (keys, then
    // op codes), their events and a copy stream, made on first use
    hipStream_t copy_stream = nullptr;
    uint8_t* feed[2] = {nullptr, nullptr};
    uint64_t feed_ops = 0;
    hipEvent_t copied[2] = {nullptr, nullptr};
    hipEvent_t consumed[2] = {nullptr, nullptr};
    bool feed_busy[2] = {false, false};
    // host-fed queries (sf_query_host): one stream, one event and one device
    // buffer (keys, then answers) per pipeline stream, made on first use
    hipStream_t qs[kMaxQueryStreams] = {};
    hipEvent_t qdone[kMaxQueryStreams] = {};
    uint8_t* qbuf[kMaxQueryStreams] = {};
    uint64_t qbuf_keys = 0;
    hipEvent_t qready = nullptr;
};

namespace {

std::mutex g_mu;
std::unordered_set<const sf_sketch*> g_live;

bool live(const sf_sketch* s) {
    std::lock_guard<std::mutex> lk(g_mu);
    return s && g_live.count(s);
}

struct Sizes {
    uint64_t fat, slim, stage, view, bpre, asnap, part, ent_key, ent_cnt, meta, hist, chunks;
    uint64_t pairs = 0, pos = 0, res = 0, level = 0, hmat = 0, pmeta = 0;  // owner path
    uint64_t base() const {
        return fat + slim + stage + view + bpre + asnap + part + ent_key + ent_cnt + meta + hist + chunks;
    }
    uint64_t owner() const { return pairs + pos + res + level + hmat + pmeta; }
    uint64_t total() const { return base() + owner(); }
};

Sizes sizes_of(const sf_config* c) {
    Sizes s;
    const uint64_t cells = uint64_t(c->d) * c->w;
    const uint64_t key = c->key_bytes == 4 ? sizeof(Key<4>) : sizeof(Key<13>);
    s.fat = round256(cells * (c->z + 1) * 4);  // the cell records
    s.slim = 0;                                 // inside the records
    s.stage = round256(cells * c->z * 4);
    s.view = round256(cells * 2);
    s.bpre = round256(uint64_t(c->d) * c->batch_ops * 4);
    s.asnap = round256(uint64_t(c->d) * c->batch_ops * 2);
    s.part = round256(uint64_t(c->batch_ops) * key);
    s.ent_key = round256(uint64_t(c->batch_ops) * key);
    s.ent_cnt = round256(uint64_t(c->batch_ops) * 4);
    s.meta = round256(sizeof(MergeMeta));
    s.hist = round256(part_groups_max(c->batch_ops, 1) * 2 * kMaxBuckets * 4);
    s.chunks = round256(merge_chunks_max(c->batch_ops) * sizeof(MergeChunk));
    OwnerGeom og;
    uint32_t lo, hi;
    if (owner_shifts(c, &lo, &hi) && owner_geom(c, &og, lo)) {  // column counts for the most ranges
        const uint64_t b = c->batch_ops, d = c->d;
        s.pairs = 2 * round256(d * b * 8);
        s.pos = round256(d * b * 4);
        s.res = round256(d * b * 8);
        s.level = round256(b * 2);
        s.hmat = round256(uint64_t(pair_tiles_max(uint32_t(b))) * og.ncol * 4);
        s.pmeta = 3 * round256(sizeof(PairMeta));
    }
    return s;
}

// The closing owner step of the pending batch, if any (before the batch that
// follows on another path, and at the end of an update call).
void close_owner(sf_sketch* s) { owner_close(&s->own, s->g, s->fat, s->slim, s->stream, &s->prof); }

// Whether a batch of cnt ops takes the owner path: each owner step reads and
// writes every record of the ranges its pairs touch, which a batch of fewer
// than w ops touches sparsely, so small batches keep the atomic entry kernels
// (measured: below about w / 2 ops per batch they are faster) unless mode 3
// asks for the owner path always.
bool use_owner(const sf_sketch* s, uint32_t cnt) { return s->owner_on && (s->owner_all || cnt >= s->cfg.w); }

// Record arrays above the 256 MiB Infinity Cache: the owner steps then wait
// on HBM, and the partition side of the next batch fills that time (measured:
// 6 % per step for 8 rows of 2^21 cells).  Smaller sketches keep one stream by
// default: their owner steps run from the cache, both sides compete for the
// same CUs, and each cross-stream wait adds several microseconds.
constexpr uint64_t kSideStreamRecords = 256ull << 20;

// Batch-wide merge: partition, merge, then S1..S5 over the entries.
template <int KB, int D>
void launch_merged(sf_sketch* s, const UniformPlan<KB>& plan, uint32_t cnt, bool ins, bool del) {
    const bool own = use_owner(s, cnt);
    if (!own) {
        close_owner(s);       // the atomic kernels read records the pending step still changes
        s->own.join = true;   // and use the merge buffers on the sketch's stream
    }
    MergeRun<KB, false> run{static_cast<MKey<KB, false>*>(s->part), static_cast<MKey<KB, false>*>(s->ent_key),
                            s->ent_cnt, s->meta, s->hist, s->chunks, s->stride, s->bpre, s->asnap, s->stride,
                            own ? &s->own : nullptr};
    run.template launch<D>(plan, blocks_for(cnt, kPartOps), cnt, OneSketch{s->g, s->fat, s->slim}, ins, del,
                           s->stream, &s->prof);
}

template <int KB>
void launch_batch(sf_sketch* s, const uint8_t* keys, const uint8_t* ops, uint32_t mode, uint32_t cnt, bool ins,
                  bool del) {
    const UniformPlan<KB> plan{keys, ops, nullptr, cnt, mode, s->g, s->fat, s->slim};
    if (s->merge_batch) {
        if (s->cfg.d == 4) launch_merged<KB, 4>(s, plan, cnt, ins, del);
        else if (s->cfg.d == 8) launch_merged<KB, 8>(s, plan, cnt, ins, del);
        else launch_merged<KB, 0>(s, plan, cnt, ins, del);
        return;
    }
    const unsigned tiles = blocks_for(cnt, uint32_t(kBlock) * s->tile_j);
    Steps<UniformPlan>::by_rows<KB>(s->cfg.d, s->tile_j, plan, tiles, ins, del, s->bpre, s->asnap, s->stride,
                                   s->stream, &s->prof, cnt);
}

enum Kind { kInsert, kDelete, kMixed };

int run_updates(sf_sketch* s, const void* keys, const uint8_t* ops, uint64_t n, Kind kind) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    if (n == 0) return SF_OK;
    const uint32_t kb = s->cfg.key_bytes;
    if (kb == 4 && (reinterpret_cast<uintptr_t>(keys) & 3u))
        return fail(SF_EINVAL, "uint32 keys must be 4-byte aligned");
    int rc = check_gpu_ptr(keys, n * kb, "keys");
    if (rc) return rc;
    if (kind == kMixed && (rc = check_gpu_ptr(ops, n, "ops"))) return rc;
    const uint8_t* k8 = static_cast<const uint8_t*>(keys);
    const uint64_t b = s->cfg.batch_ops;
    s->view_fresh = false;
    const uint32_t mode = kind == kMixed ? kOpsArray : kind == kDelete ? kAllDelete : kAllInsert;
    s->own.use_side = s->streams < 0 ? sizes_of(&s->cfg).fat > kSideStreamRecords : s->streams == 1;
    for (uint64_t lo = 0; lo < n; lo += b) {
        const uint32_t cnt = uint32_t(n - lo < b ? n - lo : b);
        const uint8_t* kp = k8 + lo * kb;
        const uint8_t* op = kind == kMixed ? ops + lo : nullptr;
        if (kb == 4) launch_batch<4>(s, kp, op, mode, cnt, kind != kDelete, kind != kInsert);
        else launch_batch<13>(s, kp, op, mode, cnt, kind != kDelete, kind != kInsert);
    }
    close_owner(s);  // the call's last batch: its S3..S5
    s->own.join = true;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = s->own.err;
    s->own.err = hipSuccess;
    return e == hipSuccess ? SF_OK : device_fail(e, "update launch");
}

template <int KB, typename S>
void query_launch(const sf_config* c, const Geom& g, const void* slim, const uint8_t* keys, uint32_t cnt,
                  uint32_t* out, hipStream_t st) {
    const UniformPlan<KB> plan{keys, nullptr, out, cnt, kAllInsert, g, nullptr, const_cast<void*>(slim)};
    launch_query_rows<KB, UniformPlan<KB>, S>(c->d, plan, blocks_for(cnt, kBlock), st);
}

// The one-row-per-XCD query over a dense uint16 Slim, with part (part_bytes
// of device scratch) holding the per-row counters of a run of keys.
int query_by_rows(Profiler* prof, const sf_config* c, const Geom& g, const uint16_t* view, const uint8_t* k8,
                  uint64_t n, uint32_t* out, uint16_t* part, uint64_t part_bytes, hipStream_t st) {
    const uint32_t kb = c->key_bytes, d = c->d;
    const uint64_t run = part_bytes / (2ull * d) < kMaxLaunch ? part_bytes / (2ull * d) : kMaxLaunch;
    for (uint64_t lo = 0; lo < n; lo += run) {
        const uint32_t cnt = uint32_t(n - lo < run ? n - lo : run);
        const uint32_t per_xcd = blocks_for(blocks_for(cnt, kBlock), kXcds / d);
        const unsigned grid = kXcds * (per_xcd < 1024u ? per_xcd : 1024u);
        const unsigned mgrid = blocks_for(cnt, kBlock) < 4096u ? blocks_for(cnt, kBlock) : 4096u;
        Timed tm(prof, st, SF_K_QUERY, cnt);
        if (kb == 4) k_query_rows<4><<<grid, kBlock, 0, st>>>(k8 + lo * kb, cnt, view, g, d, part);
        else k_query_rows<13><<<grid, kBlock, 0, st>>>(k8 + lo * kb, cnt, view, g, d, part);
        k_query_min<uint16_t><<<mgrid, kBlock, 0, st>>>(part, cnt, d, out + lo);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SF_OK : device_fail(e, "query launch");
}

int query_checks(const sf_config* c, const void* keys, uint64_t n, uint32_t* out) {
    if (c->key_bytes == 4 && (reinterpret_cast<uintptr_t>(keys) & 3u))
        return fail(SF_EINVAL, "uint32 keys must be 4-byte aligned");
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(SF_EINVAL, "out must be 4-byte aligned");
    int rc = check_gpu_ptr(keys, n * c->key_bytes, "keys");
    if (rc) return rc;
    return check_gpu_ptr(out, n * 4, "out");
}

int query_common(Profiler* prof, const sf_config* c, const Geom& g, const void* slim, bool slim16,
                 const void* keys, uint64_t n, uint32_t* out, hipStream_t st) {
    if (n == 0) return SF_OK;
    const uint32_t kb = c->key_bytes;
    if (kb == 4 && (reinterpret_cast<uintptr_t>(keys) & 3u))
        return fail(SF_EINVAL, "uint32 keys must be 4-byte aligned");
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(SF_EINVAL, "out must be 4-byte aligned");
    int rc = check_gpu_ptr(keys, n * kb, "keys");
    if (rc) return rc;
    if ((rc = check_gpu_ptr(out, n * 4, "out"))) return rc;
    const uint8_t* k8 = static_cast<const uint8_t*>(keys);
    for (uint64_t lo = 0; lo < n; lo += kMaxLaunch) {
        const uint32_t cnt = uint32_t(n - lo < kMaxLaunch ? n - lo : kMaxLaunch);
        Timed tm(prof, st, SF_K_QUERY, cnt);
        if (kb == 4) {
            if (slim16) query_launch<4, uint16_t>(c, g, slim, k8 + lo * kb, cnt, out + lo, st);
            else query_launch<4, uint32_t>(c, g, slim, k8 + lo * kb, cnt, out + lo, st);
        } else {
            if (slim16) query_launch<13, uint16_t>(c, g, slim, k8 + lo * kb, cnt, out + lo, st);
            else query_launch<13, uint32_t>(c, g, slim, k8 + lo * kb, cnt, out + lo, st);
        }
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SF_OK : device_fail(e, "query launch");
}

// The owner path's buffers (a separate allocation, so that a sketch switched
// to another merge mode gives them back).
void owner_streams_free(sf_sketch* s) {
    if (s->own.side) (void)hipStreamSynchronize(s->own.side);
    if (s->own.ev_main) (void)hipEventDestroy(s->own.ev_main);
    if (s->own.ev_p) (void)hipEventDestroy(s->own.ev_p);
    if (s->own.ev_l) (void)hipEventDestroy(s->own.ev_l);
    if (s->own.side) (void)hipStreamDestroy(s->own.side);
    s->own.side = nullptr;
    s->own.ev_main = s->own.ev_p = s->own.ev_l = nullptr;
}

int owner_alloc(sf_sketch* s) {
    const Sizes sz = sizes_of(&s->cfg);
    char* ob = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&ob), sz.owner());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "owner-path buffers: out of device memory")
                                        : device_fail(e, "owner-path buffers");
    }
    s->own_base = ob;
    s->own.pairs[0] = reinterpret_cast<uint64_t*>(ob);
    s->own.pairs[1] = reinterpret_cast<uint64_t*>(ob + sz.pairs / 2);
    s->own.pos = reinterpret_cast<uint32_t*>(ob + sz.pairs);
    s->own.cap = uint32_t(s->cfg.batch_ops);
    s->own.level_due = false;
    s->own.res = reinterpret_cast<uint64_t*>(ob + sz.pairs + sz.pos);
    s->own.level = reinterpret_cast<uint16_t*>(ob + sz.pairs + sz.pos + sz.res);
    s->own.hmat = reinterpret_cast<uint32_t*>(ob + sz.pairs + sz.pos + sz.res + sz.level);
    for (int i = 0; i < 3; i++)
        s->own.pm[i] = reinterpret_cast<PairMeta*>(ob + sz.pairs + sz.pos + sz.res + sz.level + sz.hmat +
                                                   i * (sz.pmeta / 3));
    s->own.cur = 0;
    s->own.pmc = 0;
    s->own.pending = false;
    s->own.join = true;
    if (!s->own.side) {  // the stream the partition side of the owner path runs on
        e = hipStreamCreateWithFlags(&s->own.side, hipStreamNonBlocking);  // default priority
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->own.ev_main, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->own.ev_p, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->own.ev_l, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            owner_streams_free(s);
            (void)hipFree(ob);
            s->own_base = nullptr;
            return device_fail(e, "owner-path stream");
        }
    }
    s->owner_on = true;
    return SF_OK;
}

int owner_free(sf_sketch* s) {
    s->owner_on = false;
    if (!s->own_base) return SF_OK;
    hipError_t e = hipStreamSynchronize(s->stream);  // no launch may still read them
    if (e == hipSuccess && s->own.side) e = hipStreamSynchronize(s->own.side);
    if (e == hipSuccess) e = hipFree(s->own_base);
    s->own_base = nullptr;
    return e == hipSuccess ? SF_OK : device_fail(e, "owner-path buffers free");
}

// Collector-side queries read a dense uint16 Slim one row per XCD (as
// sf_query does after an export) once it outgrows an XCD's 4 MB L2.
bool slim_by_rows(const sf_config& c) { return kXcds % c.d == 0 && uint64_t(c.d) * c.w * 2 > (4ull << 20); }

// Per-row counters one sf_query_slim run keeps in its stream-ordered scratch.
constexpr uint64_t kSlimQueryRunBytes = 32ull << 20;

int slim_query_checks(const uint16_t* slim, const sf_config* cfg, const void* keys, uint64_t n, uint32_t* out,
                      sf_config* c) {
    if (!cfg) return fail(SF_EINVAL, "null config");
    *c = *cfg;
    c->batch_ops = 1;  // not used by queries
    int rc = validate(c);
    if (rc || n == 0) return rc;
    if ((rc = check_gpu_ptr(slim, uint64_t(c->d) * c->w * 2, "slim"))) return rc;
    return query_checks(c, keys, n, out);
}

// Scratch of sf_query_slim_noalloc: the per-row counters of its one-row-per-
// XCD query.  Every GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` only names the symbol; kernels get
// the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device and kept in g_scratch.
__device__ __align__(256) uint16_t scratch[SF_NOALLOC_QUERY_COUNTERS];

std::mutex g_scratch_mu;
std::vector<uint16_t*> g_scratch;  // per device ordinal; null until looked up

int noalloc_scratch(uint16_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "sf_query_slim_noalloc device");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch.size() <= size_t(dev)) g_scratch.resize(size_t(dev) + 1, nullptr);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return device_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "sf_query_slim_noalloc scratch address");
        }
        g_scratch[dev] = static_cast<uint16_t*>(p);
    }
    *out = g_scratch[dev];
    return SF_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

uint64_t sf_footprint(const sf_config* cfg) {
    if (validate(cfg)) return 0;
    return sizes_of(cfg).total();
}

int sf_create(const sf_config* cfg, uint64_t hbm_budget_bytes, void* hip_stream, sf_sketch** out) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!out) return fail(SF_EINVAL, "null output handle");
    const Sizes sz = sizes_of(cfg);
    if (hbm_budget_bytes && sz.total() > hbm_budget_bytes)
        return fail(SF_ENOMEM, "sketch needs " + std::to_string(sz.total()) + " bytes, budget is " +
                                   std::to_string(hbm_budget_bytes));
    sf_sketch* s = new sf_sketch{};
    s->cfg = *cfg;
    s->g = geom_of(cfg);
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->stride = cfg->batch_ops;
    s->tile_j = 8;
    s->merge_batch = true;
    hipError_t e = hipGetDevice(&s->device);
    char* base = nullptr;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&base), sz.base());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "hipMalloc: out of device memory")
                                        : device_fail(e, "sf_create");
    }
    s->fat = reinterpret_cast<uint32_t*>(base);
    s->slim = reinterpret_cast<uint32_t*>(base) + cfg->z;
    s->stage = reinterpret_cast<uint16_t*>(base + sz.fat + sz.slim);
    s->stage_bytes = sz.stage;
    s->view = reinterpret_cast<uint16_t*>(base + sz.fat + sz.slim + sz.stage);
    s->view_fresh = false;
    s->bpre = reinterpret_cast<uint32_t*>(base + sz.fat + sz.slim + sz.stage + sz.view);
    s->asnap = reinterpret_cast<uint16_t*>(base + sz.fat + sz.slim + sz.stage + sz.view + sz.bpre);
    char* mq = base + sz.fat + sz.slim + sz.stage + sz.view + sz.bpre + sz.asnap;
    s->part = mq;
    s->ent_key = mq + sz.part;
    s->ent_cnt = reinterpret_cast<uint32_t*>(mq + sz.part + sz.ent_key);
    s->meta = reinterpret_cast<MergeMeta*>(mq + sz.part + sz.ent_key + sz.ent_cnt);
    s->hist = reinterpret_cast<uint32_t*>(mq + sz.part + sz.ent_key + sz.ent_cnt + sz.meta);
    s->chunks = reinterpret_cast<MergeChunk*>(mq + sz.part + sz.ent_key + sz.ent_cnt + sz.meta + sz.hist);
    s->owner_ok = owner_geom(cfg, &s->own.og);
    s->owner_on = false;
    if (s->owner_ok && (rc = owner_alloc(s))) {
        (void)hipFree(base);
        delete s;
        return rc;
    }
    e = hipMemsetAsync(s->meta, 0, sizeof(MergeMeta), s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(base, 0, sz.fat + sz.slim, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        owner_streams_free(s);
        if (s->own_base) (void)hipFree(s->own_base);
        (void)hipFree(base);
        delete s;
        return device_fail(e, "sf_create zeroing");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(s);
    }
    *out = s;
    return SF_OK;
}

int sf_destroy(sf_sketch* s) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!s || !g_live.erase(s)) return fail(SF_ESTATE, "sketch handle is not live");
    }
    hipError_t e = hipStreamSynchronize(s->stream);
    if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
    for (int i = 0; i < 2; i++) {
        if (s->feed[i]) (void)hipFree(s->feed[i]);
        if (s->copied[i]) (void)hipEventDestroy(s->copied[i]);
        if (s->consumed[i]) (void)hipEventDestroy(s->consumed[i]);
    }
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    for (uint32_t j = 0; j < kMaxQueryStreams; j++) {
        if (s->qs[j]) (void)hipStreamSynchronize(s->qs[j]);
        if (s->qbuf[j]) (void)hipFree(s->qbuf[j]);
        if (s->qdone[j]) (void)hipEventDestroy(s->qdone[j]);
        if (s->qs[j]) (void)hipStreamDestroy(s->qs[j]);
    }
    if (s->qready) (void)hipEventDestroy(s->qready);
    owner_streams_free(s);
    if (s->own_base) (void)hipFree(s->own_base);
    hipError_t e2 = hipFree(s->fat);
    delete s;
    if (e != hipSuccess) return device_fail(e, "sf_destroy sync");
    if (e2 != hipSuccess) return device_fail(e2, "sf_destroy free");
    return SF_OK;
}

int sf_reset(sf_sketch* s) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    const Sizes sz = sizes_of(&s->cfg);
    hipError_t e = hipMemsetAsync(s->fat, 0, sz.fat + sz.slim, s->stream);
    s->view_fresh = false;
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_reset");
}

int sf_set_stream(sf_sketch* s, void* hip_stream) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return device_fail(e, "sf_set_stream");
    s->stream = static_cast<hipStream_t>(hip_stream);
    return SF_OK;
}

int sf_insert(sf_sketch* s, const void* keys, uint64_t n) { return run_updates(s, keys, nullptr, n, kInsert); }

int sf_delete(sf_sketch* s, const void* keys, uint64_t n) { return run_updates(s, keys, nullptr, n, kDelete); }

int sf_update(sf_sketch* s, const void* keys, const uint8_t* ops, uint64_t n) {
    return run_updates(s, keys, ops, n, kMixed);
}

int sf_update_host(sf_sketch* s, const void* host_keys, const uint8_t* host_ops, uint64_t n, uint64_t chunk_ops) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    if (n == 0) return SF_OK;
    const uint64_t b = s->cfg.batch_ops;
    if (chunk_ops == 0 || chunk_ops % b) return fail(SF_EINVAL, "chunk_ops must be a positive multiple of batch_ops");
    auto pinned = [](const void* p) {
        hipPointerAttribute_t at{};
        if (!p || hipPointerGetAttributes(&at, p) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return at.type == hipMemoryTypeHost;
    };
    if (!pinned(host_keys)) return fail(SF_EINVAL, "host_keys must be pinned host memory (hipHostMalloc)");
    if (host_ops && !pinned(host_ops)) return fail(SF_EINVAL, "host_ops must be pinned host memory (hipHostMalloc)");
    const uint32_t kb = s->cfg.key_bytes;
    const uint64_t chunk = std::min<uint64_t>(chunk_ops, n);
    hipError_t e = hipSuccess;
    if (!s->copy_stream) {
        e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);  // default priority
        for (int i = 0; i < 2 && e == hipSuccess; i++) {
            e = hipEventCreateWithFlags(&s->copied[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s->consumed[i], hipEventDisableTiming);
        }
        if (e != hipSuccess) return device_fail(e, "sf_update_host setup");
    }
    if (s->feed_ops < chunk) {  // (re)allocate the chunk buffers once no launch reads them
        if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return device_fail(e, "sf_update_host sync");
        for (int i = 0; i < 2; i++) {
            if (s->feed[i]) (void)hipFree(s->feed[i]);
            s->feed[i] = nullptr;
            s->feed_busy[i] = false;
        }
        s->feed_ops = 0;
        for (int i = 0; i < 2; i++) {
            e = hipMalloc(reinterpret_cast<void**>(&s->feed[i]), chunk * (kb + 1));
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "sf_update_host chunk buffers")
                                                : device_fail(e, "sf_update_host chunk buffers");
            }
        }
        s->feed_ops = chunk;
    }
    const uint8_t* hk = static_cast<const uint8_t*>(host_keys);
    int last = 0;
    for (uint64_t lo = 0, c = 0; lo < n; lo += chunk, c++) {
        const int slot = int(c & 1);
        const uint64_t cnt = std::min(chunk, n - lo);
        uint8_t* dk = s->feed[slot];
        uint8_t* dop = s->feed[slot] + s->feed_ops * kb;
        // the copy into a buffer waits for the updates that read it before
        if (s->feed_busy[slot] && (e = hipStreamWaitEvent(s->copy_stream, s->consumed[slot], 0)) != hipSuccess)
            return device_fail(e, "sf_update_host wait");
        e = hipMemcpyAsync(dk, hk + lo * kb, cnt * kb, hipMemcpyHostToDevice, s->copy_stream);
        if (e == hipSuccess && host_ops)
            e = hipMemcpyAsync(dop, host_ops + lo, cnt, hipMemcpyHostToDevice, s->copy_stream);
        if (e == hipSuccess) e = hipEventRecord(s->copied[slot], s->copy_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->copied[slot], 0);
        if (e != hipSuccess) return device_fail(e, "sf_update_host copy");
        const int rc = run_updates(s, dk, host_ops ? dop : nullptr, cnt, host_ops ? kMixed : kInsert);
        if (rc) return rc;
        if ((e = hipEventRecord(s->consumed[slot], s->stream)) != hipSuccess)
            return device_fail(e, "sf_update_host record");
        s->feed_busy[slot] = true;
        last = slot;
    }
    // every byte has left the host buffers once the last copy is done
    e = hipEventSynchronize(s->copied[last]);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_update_host copies");
}

int sf_query_host(sf_sketch* s, const void* host_keys, uint64_t n, uint32_t* host_out, uint32_t streams) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    if (streams < 1 || streams > kMaxQueryStreams) return fail(SF_EINVAL, "streams must be in 1..16");
    if (n == 0) return SF_OK;
    auto pinned = [](const void* p) {
        hipPointerAttribute_t at{};
        if (!p || hipPointerGetAttributes(&at, p) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return at.type == hipMemoryTypeHost;
    };
    if (!pinned(host_keys)) return fail(SF_EINVAL, "host_keys must be pinned host memory (hipHostMalloc)");
    if (!pinned(host_out)) return fail(SF_EINVAL, "host_out must be pinned host memory (hipHostMalloc)");
    const uint32_t kb = s->cfg.key_bytes;
    const uint64_t share = n / streams + (n % streams ? 1 : 0);  // the largest share
    hipError_t e = hipSuccess;
    if (!s->qready && (e = hipEventCreateWithFlags(&s->qready, hipEventDisableTiming)) != hipSuccess)
        return device_fail(e, "sf_query_host setup");
    if (s->qbuf_keys < share) {  // (re)allocate the per-stream buffers once nothing reads them
        for (uint32_t j = 0; j < kMaxQueryStreams; j++) {
            if (s->qs[j] && (e = hipStreamSynchronize(s->qs[j])) != hipSuccess)
                return device_fail(e, "sf_query_host sync");
            if (s->qbuf[j]) (void)hipFree(s->qbuf[j]);
            s->qbuf[j] = nullptr;
        }
        s->qbuf_keys = 0;
    }
    for (uint32_t j = 0; j < streams; j++) {
        if (!s->qs[j]) {
            e = hipStreamCreateWithFlags(&s->qs[j], hipStreamNonBlocking);  // default priority
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s->qdone[j], hipEventDisableTiming);
            if (e != hipSuccess) return device_fail(e, "sf_query_host streams");
        }
        if (!s->qbuf[j]) {
            e = hipMalloc(reinterpret_cast<void**>(&s->qbuf[j]), std::max<uint64_t>(share, s->qbuf_keys) * (kb + 4) + 4);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "sf_query_host buffers")
                                                : device_fail(e, "sf_query_host buffers");
            }
        }
    }
    s->qbuf_keys = std::max<uint64_t>(s->qbuf_keys, share);
    // every stream starts after the work already on the sketch's stream
    if ((e = hipEventRecord(s->qready, s->stream)) != hipSuccess) return device_fail(e, "sf_query_host record");
    // the one-pass query (the row split's scratch is the sketch's own, one at a time)
    const void* slim = s->view_fresh ? static_cast<const void*>(s->view) : static_cast<const void*>(s->slim);
    const uint8_t* hk = static_cast<const uint8_t*>(host_keys);
    const uint64_t base = n / streams, extra = n % streams;
    uint64_t off = 0;
    for (uint32_t j = 0; j < streams; j++) {
        const uint64_t cnt = base + (j < extra ? 1 : 0);  // the first n mod streams take one more
        if (!cnt) continue;
        uint8_t* dk = s->qbuf[j];
        uint32_t* dout = reinterpret_cast<uint32_t*>(s->qbuf[j] + ((s->qbuf_keys * kb + 3) & ~uint64_t(3)));
        e = hipStreamWaitEvent(s->qs[j], s->qready, 0);
        if (e == hipSuccess) e = hipMemcpyAsync(dk, hk + off * kb, cnt * kb, hipMemcpyHostToDevice, s->qs[j]);
        if (e != hipSuccess) return device_fail(e, "sf_query_host copy in");
        int rc = query_common(&s->prof, &s->cfg, s->g, slim, s->view_fresh, dk, cnt, dout, s->qs[j]);
        if (rc) return rc;
        e = hipMemcpyAsync(host_out + off, dout, cnt * 4, hipMemcpyDeviceToHost, s->qs[j]);
        if (e == hipSuccess) e = hipEventRecord(s->qdone[j], s->qs[j]);
        // later work on the sketch's stream (updates, resets) waits for these reads
        if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->qdone[j], 0);
        if (e != hipSuccess) return device_fail(e, "sf_query_host copy out");
        off += cnt;
    }
    for (uint32_t j = 0; j < streams; j++)
        if (base + (j < extra ? 1 : 0) && (e = hipEventSynchronize(s->qdone[j])) != hipSuccess)
            return device_fail(e, "sf_query_host wait");
    return SF_OK;
}

int sf_query(sf_sketch* s, const void* keys, uint64_t n, uint32_t* out) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    // the dense uint16 Slim, one row per XCD, once the whole copy outgrows an
    // XCD's 4 MB L2
    if (s->view_fresh && kXcds % s->cfg.d == 0 && uint64_t(s->cfg.d) * s->cfg.w * 2 > (4ull << 20)) {
        if (n == 0) return SF_OK;
        int rc = query_checks(&s->cfg, keys, n, out);
        if (rc) return rc;
        return query_by_rows(&s->prof, &s->cfg, s->g, s->view, static_cast<const uint8_t*>(keys), n, out,
                             reinterpret_cast<uint16_t*>(s->stage), s->stage_bytes, s->stream);
    }
    if (s->view_fresh)  // the dense uint16 Slim: a fifth of the records' footprint
        return query_common(&s->prof, &s->cfg, s->g, s->view, true, keys, n, out, s->stream);
    return query_common(&s->prof, &s->cfg, s->g, s->slim, false, keys, n, out, s->stream);
}

int sf_query_slim(const uint16_t* slim, const sf_config* cfg, const void* keys, uint64_t n, uint32_t* out,
                  void* hip_stream) {
    sf_config c{};
    int rc = slim_query_checks(slim, cfg, keys, n, out, &c);
    if (rc || n == 0) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (!slim_by_rows(c)) return query_common(nullptr, &c, geom_of(&c), slim, true, keys, n, out, st);
    // per-row counters of a run of keys, in stream-ordered scratch freed behind the run
    const uint64_t run = std::min<uint64_t>(n, kSlimQueryRunBytes / (2ull * c.d));
    void* part = nullptr;
    hipError_t e = hipMallocAsync(&part, run * c.d * 2, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "sf_query_slim scratch") : device_fail(e, "sf_query_slim scratch");
    }
    rc = query_by_rows(nullptr, &c, geom_of(&c), slim, static_cast<const uint8_t*>(keys), n, out,
                       static_cast<uint16_t*>(part), run * c.d * 2, st);
    e = hipFreeAsync(part, st);
    if (rc) return rc;
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_query_slim scratch free");
}

int sf_query_slim_noalloc(const uint16_t* slim, const sf_config* cfg, const void* keys, uint64_t n, uint32_t* out,
                          void* hip_stream) {
    sf_config c{};
    int rc = slim_query_checks(slim, cfg, keys, n, out, &c);
    if (rc || n == 0) return rc;
    if (n * c.d > SF_NOALLOC_QUERY_COUNTERS)
        return fail(SF_EINVAL, "sf_query_slim_noalloc: n * d = " + std::to_string(n * c.d) +
                                   " per-row counters exceed its static scratch of " +
                                   std::to_string(SF_NOALLOC_QUERY_COUNTERS) + "; split the keys over several calls");
    uint16_t* part = nullptr;
    if ((rc = noalloc_scratch(&part))) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (!slim_by_rows(c)) return query_common(nullptr, &c, geom_of(&c), slim, true, keys, n, out, st);
    return query_by_rows(nullptr, &c, geom_of(&c), slim, static_cast<const uint8_t*>(keys), n, out, part,
                         uint64_t(SF_NOALLOC_QUERY_COUNTERS) * 2, st);
}

int sf_export_slim(sf_sketch* s, uint16_t* out, uint64_t out_elems) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    const uint64_t cells = uint64_t(s->cfg.d) * s->cfg.w;
    if (!out) return fail(SF_EINVAL, "out is null");
    if (out_elems < cells) return fail(SF_EINVAL, "out_elems < d*w");
    const bool host = host_dest(out);
    if (!host) {
        int rc = check_gpu_ptr(out, cells * 2, "out");
        if (rc) return rc;
    }
    const unsigned grid = blocks_for(cells, kBlock) < 4096u ? blocks_for(cells, kBlock) : 4096u;
    hipError_t e = hipSuccess;
    if (!s->view_fresh) {  // pack the records' Slim words into the view and (device) out at once
        Timed tm(&s->prof, s->stream, SF_K_EXPORT, cells);
        k_pack16<uint32_t><<<dim3(grid), dim3(kBlock), 0, s->stream>>>(s->slim, s->view, cells, s->g.rs,
                                                                       host ? nullptr : out);
        e = hipGetLastError();
        s->view_fresh = e == hipSuccess;
    } else if (!host) {
        e = hipMemcpyAsync(out, s->view, cells * 2, hipMemcpyDeviceToDevice, s->stream);
    }
    // a host destination is complete on return; a device one is written in
    // order on the sketch's stream, like every other device output
    if (e == hipSuccess && host) e = hipMemcpyAsync(out, s->view, cells * 2, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && host) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_export_slim");
}

int sf_export_fat(sf_sketch* s, uint32_t* out, uint64_t out_elems) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    const uint64_t n = uint64_t(s->cfg.d) * s->cfg.w * s->cfg.z;
    if (!out) return fail(SF_EINVAL, "out is null");
    if (out_elems < n) return fail(SF_EINVAL, "out_elems < d*w*z");
    const bool host = host_dest(out);
    if (!host) {
        int rc = check_gpu_ptr(out, n * 4, "out");
        if (rc) return rc;
    }
    uint32_t* dst = host ? reinterpret_cast<uint32_t*>(s->stage) : out;
    const uint64_t cells = uint64_t(s->cfg.d) * s->cfg.w;
    const unsigned grid = blocks_for(n, kBlock) < 4096u ? blocks_for(n, kBlock) : 4096u;
    k_unpack_fat<uint32_t><<<dim3(grid), dim3(kBlock), 0, s->stream>>>(s->fat, dst, cells, s->cfg.z);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && host) e = hipMemcpyAsync(out, dst, n * 4, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_export_fat");
}

int sf_sync(sf_sketch* s) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess && s->own.side) e = hipStreamSynchronize(s->own.side);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_sync");
}

int sf_set_tile(sf_sketch* s, uint32_t tile_ops) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    if (tile_ops != 256 && tile_ops != 1024 && tile_ops != 2048)
        return fail(SF_EINVAL, "tile_ops must be 256, 1024 or 2048");
    s->tile_j = tile_ops / kBlock;
    return SF_OK;
}

int sf_set_merge(sf_sketch* s, int batch_wide) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    if (batch_wide < 0 || batch_wide > 3) return fail(SF_EINVAL, "merge mode must be 0, 1, 2 or 3");
    s->merge_batch = batch_wide != 0;
    s->owner_all = batch_wide == 3;
    if ((batch_wide == 1 || batch_wide == 3) && s->owner_ok)
        return s->own_base ? (s->owner_on = true, SF_OK) : owner_alloc(s);
    return owner_free(s);
}

int sf_set_owner_range(sf_sketch* s, uint32_t shift) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    if (!s->owner_ok) return fail(SF_EINVAL, "this sketch shape has no owner-computes path");
    OwnerGeom og;
    if (!owner_geom(&s->cfg, &og, shift)) {
        uint32_t lo = 0, hi = 0;
        owner_shifts(&s->cfg, &lo, &hi);
        return fail(SF_EINVAL, "range shift must be 0 or within [" + std::to_string(lo) + ", " +
                                   std::to_string(hi) + "] for this shape");
    }
    s->own.og = og;  // launches already queued keep the layout they were given
    return SF_OK;
}

int sf_owner_range(sf_sketch* s) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    return s->owner_ok ? int(s->own.og.cr_shift) : 0;
}

int sf_set_streams(sf_sketch* s, int mode) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    if (mode < -1 || mode > 1) return fail(SF_EINVAL, "streams mode must be -1, 0 or 1");
    s->streams = mode;
    return SF_OK;
}

int sf_merge_path(sf_sketch* s) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    return !s->merge_batch ? 0 : !s->owner_on ? 2 : s->owner_all ? 3 : 1;
}

int sf_merge_stats(sf_sketch* s, uint64_t* insert_entries, uint64_t* delete_entries) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    unsigned long long acc[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(acc, &s->meta->acc_ins, sizeof(acc), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return device_fail(e, "sf_merge_stats");
    if (insert_entries) *insert_entries = acc[0];
    if (delete_entries) *delete_entries = acc[1];
    return SF_OK;
}

int sf_profile(sf_sketch* s, int enable) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    s->prof.on = enable != 0;
    return SF_OK;
}

int sf_profile_read(sf_sketch* s, sf_kernel_stats* out, int reset) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    int rc = s->prof.drain();
    if (out) *out = s->prof.acc;
    if (reset) s->prof.acc = sf_kernel_stats{};
    return rc;
}

const char* sf_strerror(int status) {
    switch (status) {
        case SF_OK: return "ok";
        case SF_EINVAL: return "invalid argument";
        case SF_ENOMEM: return "out of memory or over the HBM budget";
        case SF_EDEVICE: return "HIP device error";
        case SF_ESTATE: return "handle is not live";
        case SF_EUNDERFLOW: return "delete of an absent item (strict-turnstile violation)";
        default: return "unknown status";
    }
}

const char* sf_last_error(void) { return last_error().c_str(); }

}  // extern "C"
