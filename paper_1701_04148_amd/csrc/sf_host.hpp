// Host-side helpers shared by the single-sketch and sketch-group entry
// points: error reporting, config validation, pointer checks, geometry,
// launch dispatch and per-kernel event timing.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sf.h"
#include "sf_owner.hpp"

namespace sfh {

using namespace sfk;

std::string& last_error();  // thread-local detail string (defined in sf_lib.hip)

inline int fail(int code, const std::string& msg) {
    last_error() = msg;
    return code;
}

inline int device_fail(hipError_t e, const char* what) {
    return fail(SF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr uint64_t kMaxBatch = 1ull << 30;
constexpr uint32_t kMaxLaunch = 1u << 30;  // ops per kernel launch (uint32 indexing)

inline bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

inline int validate(const sf_config* c) {
    if (!c) return fail(SF_EINVAL, "null config");
    if (c->d < 1 || c->d > uint32_t(kMaxD)) return fail(SF_EINVAL, "d must be in 1..16");
    if (c->w < 1 || c->z < 1) return fail(SF_EINVAL, "w and z must be >= 1");
    if (uint64_t(c->w) * c->z > (1ull << 32)) return fail(SF_EINVAL, "w*z must be <= 2^32");
    if (c->key_bytes != 4 && c->key_bytes != 13) return fail(SF_EINVAL, "key_bytes must be 4 or 13");
    if (c->batch_ops < 1 || c->batch_ops > kMaxBatch) return fail(SF_EINVAL, "batch_ops must be in 1..2^30");
    return SF_OK;
}

inline uint64_t round256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

inline Geom geom_of(const sf_config* c) {
    Geom g{};
    g.d = c->d;
    g.w = c->w;
    g.z = c->z;
    g.rs = c->z + 1;
    g.seed_base = c->seed_base;
    const uint64_t wz = uint64_t(c->w) * c->z;
    g.wz32 = uint32_t(wz);  // 2^32 wraps to 0
    g.pow2 = is_pow2(c->w) && is_pow2(c->z);
    if (g.pow2) {
        g.w_mask = c->w - 1;
        g.wz_mask = uint32_t(wz - 1);
        g.w_shift = uint32_t(__builtin_ctzll(c->w));
    }
    return g;
}

// A pointer the GPU may read or write: device memory (checked to hold
// `bytes` from p on) or pinned host memory.  Rejects pageable host memory,
// which a kernel cannot touch.
inline int check_gpu_ptr(const void* p, uint64_t bytes, const char* what) {
    if (!p) return fail(SF_EINVAL, std::string(what) + " is null");
    hipPointerAttribute_t at{};
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SF_EINVAL, std::string(what) + " is not GPU-accessible memory");
    }
    if (at.type == hipMemoryTypeDevice) {
        void* base = nullptr;
        size_t size = 0;
        if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && base) {
            const uint64_t off = uint64_t(static_cast<const char*>(p) - static_cast<const char*>(base));
            if (off + bytes > size)
                return fail(SF_EINVAL, std::string(what) + " buffer is smaller than the requested size");
        } else {
            (void)hipGetLastError();
        }
        return SF_OK;
    }
    if (at.type == hipMemoryTypeHost || at.isManaged) return SF_OK;
    return fail(SF_EINVAL, std::string(what) + " is not GPU-accessible memory");
}

inline bool host_dest(void* p) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return at.type != hipMemoryTypeDevice && !at.isManaged;
}

inline unsigned blocks_for(uint64_t n, uint32_t per_block) { return unsigned((n + per_block - 1) / per_block); }

// ---------------------------------------------------------------- timing
// Brackets launches with HIP events on the launching stream when enabled.
struct Profiler {
    struct Rec {
        int kind;
        uint64_t items;
        hipEvent_t a, b;
    };
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    sf_kernel_stats acc{};

    hipEvent_t take() {
        hipEvent_t e = nullptr;
        if (!spare.empty()) {
            e = spare.back();
            spare.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }

    int drain() {
        hipError_t err = hipSuccess;
        for (auto& r : recs) {
            float ms = 0.f;
            hipError_t e = hipEventSynchronize(r.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
            if (e != hipSuccess && err == hipSuccess) err = e;
            acc.ms[r.kind] += ms;
            acc.launches[r.kind] += 1;
            acc.items[r.kind] += r.items;
            spare.push_back(r.a);
            spare.push_back(r.b);
        }
        recs.clear();
        return err == hipSuccess ? SF_OK : device_fail(err, "profile events");
    }

    ~Profiler() {
        for (auto& r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : spare) (void)hipEventDestroy(e);
    }
};

struct Timed {
    Profiler* p;
    hipStream_t st;
    Profiler::Rec r;
    Timed(Profiler* prof, hipStream_t stream, int kind, uint64_t items)
        : p(prof && prof->on ? prof : nullptr), st(stream), r{kind, items, nullptr, nullptr} {
        if (!p) return;
        r.a = p->take();
        r.b = p->take();
        if (r.a) (void)hipEventRecord(r.a, st);
    }
    ~Timed() {
        if (!p || !r.a || !r.b) return;
        (void)hipEventRecord(r.b, st);
        p->recs.push_back(r);
    }
};

// ---------------------------------------------------------------- launches
// The five steps of one schedule batch (or round of a group) over plan P.
template <int KB, int D, int J, class P>
void launch_steps(const P& plan, unsigned tiles, bool ins, bool del, uint32_t* bpre, uint16_t* asnap,
                  uint32_t stride, hipStream_t st, Profiler* prof, uint64_t items) {
    const dim3 grid(tiles), block(kBlock);
    if (ins) {
        {
            Timed tm(prof, st, SF_K_SNAPSHOT, items);
            k_snapshot<KB, D, J, P><<<grid, block, 0, st>>>(plan, bpre, asnap, stride);
        }
        {
            Timed tm(prof, st, SF_K_FAT_ADD, items);
            k_fat_update<KB, D, J, P><<<grid, block, 0, st>>>(plan, 0u);
        }
        {
            Timed tm(prof, st, SF_K_RAISE, items);
            k_raise<KB, D, J, P><<<grid, block, 0, st>>>(plan, bpre, asnap, stride);
        }
    }
    if (del) {
        {
            Timed tm(prof, st, SF_K_FAT_SUB, items);
            k_fat_update<KB, D, J, P><<<grid, block, 0, st>>>(plan, 1u);
        }
        {
            Timed tm(prof, st, SF_K_CLAMP, items);
            k_clamp<KB, D, J, P><<<grid, block, 0, st>>>(plan);
        }
    }
}

// Range sizes of the owner-computes path for a sketch shape: 2^shift cells,
// from the smallest shift (at least 4) that keeps a row at most kMaxRanges
// ranges and the columns of both op types within kMaxCols, up to the largest
// whose Fat counters fit the owners' LDS and a pair's 16-bit local code.  The
// shape qualifies when the smallest is within that limit.
inline bool owner_shifts(const sf_config* c, uint32_t* lo, uint32_t* hi) {
    const uint32_t rmax = std::min<uint32_t>(kMaxRanges, kMaxCols / (2 * c->d));
    uint32_t zbits = 0;
    while ((1ull << zbits) < c->z) zbits++;
    uint32_t sh = 4;
    while (((uint64_t(c->w) + (1ull << sh) - 1) >> sh) > rmax) sh++;
    auto fits = [&](uint32_t x) { return (1ull << x) * c->z <= kOwnCounters && ((1ull << x) << zbits) <= 65536; };
    if (!fits(sh)) return false;
    *lo = sh;
    while (fits(sh + 1) && (1ull << sh) < c->w) sh++;
    *hi = sh;
    return true;
}

// Default range size: about kDefaultRanges ranges per row, at least 256
// cells (fewer, busier owner workgroups and a shorter column scan for narrow
// sketches), within the allowed sizes.  (Measured: 2048-cell ranges at
// w = 2^20, 256 at w = 2^14.)
constexpr uint32_t kDefaultRangeShiftMin = 8, kDefaultRangesLog2 = 9;

// The owner layout with ranges of 2^shift cells (0: the default size).
inline bool owner_geom(const sf_config* c, OwnerGeom* og, uint32_t shift = 0) {
    uint32_t lo, hi;
    if (!owner_shifts(c, &lo, &hi)) return false;
    uint32_t wl = 0;
    while ((1ull << (wl + 1)) <= c->w) wl++;  // floor(log2 w)
    const uint32_t want = std::max(kDefaultRangeShiftMin, wl > kDefaultRangesLog2 ? wl - kDefaultRangesLog2 : 0u);
    const uint32_t sh = shift ? shift : std::min(hi, std::max(lo, want));
    if (sh < lo || sh > hi) return false;
    uint32_t zbits = 0;
    while ((1ull << zbits) < c->z) zbits++;
    const uint64_t cr = 1ull << sh;
    og->R = uint32_t((uint64_t(c->w) + cr - 1) >> sh);
    og->cr_shift = sh;
    og->zbits = zbits;
    og->ncol = 2 * c->d * og->R;
    og->xcd = (kXcds % c->d == 0 && (c->d * og->R) % kXcds == 0) ? 1u : 0u;
    og->d = c->d;
    return true;
}

// Device buffers of the owner-computes path (cap = entry capacity = b).  A
// batch's S3..S5 run in the owner step of the next batch of the same update
// call (or in a closing step), so the pairs and column starts of two batches
// are alive at once: set `cur` takes the next batch, set cur ^ 1 holds the
// batch whose S3..S5 are pending.
struct OwnerBufs {
    OwnerGeom og;
    uint64_t* pairs[2];  // [d * cap] pairs, in column order
    PairMeta* pm[3];     // column starts (a sketch table uses set 0 only)
    uint32_t* pos;       // [d][cap] position of each insert entry's pair per row
    uint64_t* res;       // [d * cap] per insert pair: Slim before, growth, Fat after (16 bits each)
    uint16_t* level;     // [cap] T of each insert entry
    uint32_t* hmat;      // [pair_tiles_max(cap)][ncol] per-tile column counts, then offsets
    uint32_t cur = 0;    // pairs set of the next batch
    uint32_t pmc = 0;    // column-start set of the next batch
    bool pending = false;
    // Lone sketch: the partition, merge and pair kernels run on `side` (when
    // set), the owner steps and k_level on the sketch's stream.
    hipStream_t side = nullptr;
    hipEvent_t ev_main = nullptr;  // the sketch's stream up to here (side waits before its next batch)
    hipEvent_t ev_p = nullptr;     // a batch's pairs written (the sketch's stream waits)
    hipEvent_t ev_l = nullptr;     // a batch's k_level done (side waits before writing pairs and pos)
    bool use_side = false;         // run the partition side there (set per update call)
    bool join = true;              // side must first wait for the sketch's stream
    bool l_rec = false;            // ev_l holds the previous batch's k_level
    hipError_t err = hipSuccess;   // first failed event call since the last check
    void mark(hipError_t e) {
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
    // One stream: a batch's k_level waits to share a launch with the next
    // batch's k_part_count; level_flush launches it alone (call end, path
    // switch).
    bool level_due = false;
    uint32_t level_pset = 0, level_tiles = 0, cap = 0;
    const void* level_keys = nullptr;
    void (*level_flush)(OwnerBufs*, hipStream_t) = nullptr;
};

// k_level of the deferred batch on its own.
template <int D, int KB>
void flush_level(OwnerBufs* o, hipStream_t st) {
    k_level<D, KB, false, LoneRanges><<<o->level_tiles, kPairThreads, 0, st>>>(
        o->pm[o->level_pset], static_cast<const MKey<KB, false>*>(o->level_keys), LoneRanges{}, o->pos, o->cap,
        o->res, o->og.d, o->level);
    o->level_due = false;
}

// LDS of one owner step: the range's records.
inline size_t own_step_lds(const Geom& g, const OwnerGeom& og) {
    return (size_t(1) << og.cr_shift) * g.rs * 4;
}

// One owner-step launch: 512-thread workgroups for ranges of more than
// kOwnWideLds bytes (fewer of them fit a CU, so each gets more waves).
template <class SR, class RM>
inline void launch_own_step(unsigned grid, size_t lds, hipStream_t st, const SR& sr, const RM& rm,
                            const OwnerGeom& og, const PairMeta* pm_f, const uint64_t* pairs_f,
                            const uint16_t* level, const PairMeta* pm_i, const uint64_t* pairs_i, uint64_t* res) {
    if (lds > kOwnWideLds)
        k_own_step<SR, RM, kOwnThreadsWide><<<grid, kOwnThreadsWide, lds, st>>>(sr, rm, og, pm_f, pairs_f, level,
                                                                                pm_i, pairs_i, res);
    else
        k_own_step<SR, RM><<<grid, kOwnThreads, lds, st>>>(sr, rm, og, pm_f, pairs_f, level, pm_i, pairs_i, res);
}

// The closing owner step of an update call: S3..S5 of its last batch.
inline void owner_close(OwnerBufs* own, const Geom& g, uint32_t* fat, uint32_t* slim, hipStream_t st,
                        Profiler* prof) {
    if (own->level_due) own->level_flush(own, st);
    if (!own->pending) return;
    const uint32_t prev = own->cur ^ 1u, pprev = (own->pmc + 2u) % 3u;
    Timed tm(prof, st, SF_K_OWN_FINAL, 0);
    launch_own_step(g.d * own->og.R, own_step_lds(g, own->og), st, OneSketch{g, fat, slim}, LoneRanges{}, own->og,
                    own->pm[pprev], own->pairs[prev], own->level, nullptr, nullptr, own->res);
    own->pending = false;
}

// Dispatch of (key width, rows, tile) to kernel instantiations.
// The batch-merge path of one schedule batch (or round): partition the ops
// into hash buckets, merge each bucket chunk in LDS into entries, then S1..S5
// once per entry.  G: the merged key carries its sketch's index.
template <int KB, bool G>
struct MergeRun {
    MKey<KB, G>* part;     // [cap] partitioned keys
    MKey<KB, G>* ent_key;  // [cap] entries: inserts from 0 up, deletes from cap-1 down
    uint32_t* ent_cnt;     // [cap]
    MergeMeta* meta;
    uint32_t* hist;        // [part groups][2 * kMaxBuckets] per-group bucket histograms / offsets
    MergeChunk* chunks;    // [merge_chunks_max(cap)] key range of every merge chunk
    uint32_t cap;
    uint32_t* bpre;        // [d][stride] S1 snapshot of Fat counters, per insert entry
    uint16_t* asnap;       // [d][stride] S1 snapshot of Slim counters, per insert entry
    uint32_t stride;
    OwnerBufs* own = nullptr;  // S1..S5 by (row, cell range) owners
    // a sketch table's sub-round: its ranges and their layout (own set)
    TableRanges sub_rm{};
    OwnerGeom sub_og{};
    uint32_t max_z = 0;
    bool side_atomic = false;  // ... some of whose sketches take the atomic entry kernels

    template <int D, class SR>
    void launch_owner(uint32_t cnt, const SR& sr, bool ins, bool del, hipStream_t st, hipStream_t ps,
                      Profiler* prof) const;
    template <class SR, class RM>
    void launch_pairs(uint32_t cnt, const SR& sr, const RM& rm, const OwnerGeom& og, uint32_t set, uint32_t pset,
                      hipStream_t st, Profiler* prof, hipEvent_t before_scatter = nullptr) const;

    // part_groups: workgroups of the partition kernels (plan tiles of at most
    // kPartOps ops); cnt: ops in the batch (<= cap).
    template <int D, class P, class SR>
    void launch(const P& plan, unsigned part_groups, uint32_t cnt, const SR& sr, bool ins, bool del,
                hipStream_t st, Profiler* prof) const {
        const uint32_t nb = buckets_for<KB, G>(cnt);
        const uint32_t nb_log2 = uint32_t(__builtin_ctz(nb));
        const unsigned eg = blocks_for(cnt, kBlock) < 4096u ? blocks_for(cnt, kBlock) : 4096u;
        // S1 one row per XCD when the row count divides the XCD count: the same
        // threads per row as eg per entry, in a multiple of 8 workgroups
        const unsigned xg = kXcds * (blocks_for(uint64_t(eg) * (D > 0 ? D : 1), kXcds) < 1024u
                                         ? blocks_for(uint64_t(eg) * (D > 0 ? D : 1), kXcds)
                                         : 1024u);
        // A lone sketch's owner path runs partition, merge and pairs on the side
        // stream (not while profiling: the per-kind events then time one stream)
        hipStream_t ps = st;
        if (!G && own && own->side && own->use_side && !(prof && prof->on)) {
            ps = own->side;
            if (own->join) {  // the keys (and everything before) are the sketch stream's
                own->mark(hipEventRecord(own->ev_main, st));
                own->mark(hipStreamWaitEvent(ps, own->ev_main, 0));
                own->join = false;
                own->l_rec = false;
            }
        } else if (own) {
            own->join = true;
        }
        // a lone sketch's large batches of uint32 keys: tiles of kPartOpsWide
        // ops (the staged keys of one still fit the LDS), so that every bucket's
        // run is longer; smaller batches keep more, smaller tiles
        constexpr bool kWideOk = !G && KB == 4;
        const bool wide = kWideOk && cnt >= kWideBatch;
        if (wide) part_groups = blocks_for(cnt, kPartOpsWide);
        {
            Timed tm(prof, ps, SF_K_PARTITION, cnt);
            bool counted = false;
            if constexpr (!G) {
                // the previous batch's k_level rides along (one stream only)
                if (own && own->level_due && ps == st) {
                    const unsigned grid = part_groups + own->level_tiles;
                    if (wide)
                        k_part_count_level<KB, P, kPartOpsWide, D><<<grid, kPartThreads, 0, ps>>>(
                            plan, hist, nb_log2, part_groups, own->pm[own->level_pset], ent_key, own->pos, cap,
                            own->res, own->og.d, own->level);
                    else
                        k_part_count_level<KB, P, kPartOps, D><<<grid, kPartThreads, 0, ps>>>(
                            plan, hist, nb_log2, part_groups, own->pm[own->level_pset], ent_key, own->pos, cap,
                            own->res, own->og.d, own->level);
                    own->level_due = false;
                    counted = true;
                } else if (own && own->level_due) {
                    own->level_flush(own, st);
                }
            }
            if (counted) {
            } else if (wide)
                k_part_count<KB, G, P, kPartOpsWide><<<part_groups, kPartThreads, 0, ps>>>(plan, hist, nb_log2);
            else
                k_part_count<KB, G, P><<<part_groups, kPartThreads, 0, ps>>>(plan, hist, nb_log2);
            // one lane per bucket pays off for 256..1024 rows; fewer rows (small
            // batches) or more (sketch tables) spread better over segments
            if (part_groups >= kScanWaves * kScanRowsReg / 4 && part_groups <= kScanWaves * kScanRowsReg)
                k_part_colscan<uint32_t><<<blocks_for(2 * nb, kScanCols), kScanCols * kScanWaves, 0, ps>>>(
                    hist, part_groups, 2 * nb, meta);
            else
                k_part_colscan_tall<uint32_t><<<blocks_for(2 * nb, kScanBuckets), kScanBuckets * kScanSegs, 0, ps>>>(
                    hist, part_groups, 2 * nb, meta);
            bool done = false;
            if constexpr (!G) {
                // all buckets in use: the layout workgroup rides in the scatter launch
                if (nb == kMaxBuckets) {
                    if (wide)
                        k_part_scatter_start<KB, P, kPartOpsWide><<<part_groups + 1, kPartThreads, 0, ps>>>(
                            plan, hist, meta, chunks, part, nb_log2, part_groups);
                    else
                        k_part_scatter_start<KB, P, kPartOps><<<part_groups + 1, kPartThreads, 0, ps>>>(
                            plan, hist, meta, chunks, part, nb_log2, part_groups);
                    done = true;
                }
            }
            if (!done) {
                k_part_start<KB, G><<<1, 2 * nb / kStartPer, 0, ps>>>(meta, chunks);
                if constexpr (kWideOk) {
                    if (wide) {
                        k_part_scatter<KB, G, P, kPartOpsWide><<<part_groups, kPartThreads, 0, ps>>>(
                            plan, hist, meta, part, nb_log2);
                        done = true;
                    }
                }
                if (!done)
                    k_part_scatter<KB, G, P><<<part_groups, kPartThreads, 0, ps>>>(plan, hist, meta, part, nb_log2);
            }
        }
        {
            Timed tm(prof, ps, SF_K_MERGE, cnt);
            k_merge<KB, G, SR><<<blocks_for(cnt, MergeShape<KB, G>::kChunk) + 2 * nb, MergeShape<KB, G>::kThreads, 0,
                                 ps>>>(part, meta, chunks, ent_key, ent_cnt, cap, nb_log2, sr, bpre, asnap,
                                       own ? 0u : 1u);
        }
        if (own) {
            if constexpr (G) {
                // a sub-round whose sparse sketches keep the atomic path: their
                // entries first (SketchSide skips the owner-computed sketches)
                if (side_atomic)
                    launch_entries<D>(eg, xg, cnt, SketchSide{sr.t, sub_rm.qbase}, ins, del, st, prof);
            }
            launch_owner<D>(cnt, sr, ins, del, st, ps, prof);
            return;
        }
        launch_entries<D>(eg, xg, cnt, sr, ins, del, st, prof);
    }

    // S1..S5 with one device-scope atomic per entry and row (the entries sr takes).
    template <int D, class SR>
    void launch_entries(unsigned eg, unsigned xg, uint32_t cnt, const SR& sr, bool ins, bool del, hipStream_t st,
                        Profiler* prof) const {
        constexpr bool kRowsPerXcd = D > 0 && kXcds % (D > 0 ? D : 1) == 0;
        if (ins) {
            {
                Timed tm(prof, st, SF_K_SNAPSHOT, cnt);
                if constexpr (kRowsPerXcd)
                    k_entries_snapshot_rows<KB, D, G, SR><<<xg, kBlock, 0, st>>>(meta, ent_key, ent_cnt, sr, bpre,
                                                                                 asnap, stride);
                else
                    k_entries_snapshot<KB, D, G, SR><<<eg, kBlock, 0, st>>>(meta, ent_key, ent_cnt, sr, bpre, asnap,
                                                                            stride);
            }
            {
                Timed tm(prof, st, SF_K_FAT_ADD, cnt);
                k_entries_fat<KB, D, G, SR><<<eg, kBlock, 0, st>>>(meta, ent_key, ent_cnt, cap, sr, 0u);
            }
            {
                Timed tm(prof, st, SF_K_RAISE, cnt);
                k_entries_raise<KB, D, G, SR><<<eg, kBlock, 0, st>>>(meta, ent_key, sr, bpre, asnap, stride);
            }
        }
        if (del) {
            {
                Timed tm(prof, st, SF_K_FAT_SUB, cnt);
                k_entries_fat<KB, D, G, SR><<<eg, kBlock, 0, st>>>(meta, ent_key, ent_cnt, cap, sr, 1u);
            }
            {
                Timed tm(prof, st, SF_K_CLAMP, cnt);
                k_entries_clamp<KB, D, G, SR><<<eg, kBlock, 0, st>>>(meta, ent_key, cap, sr);
            }
        }
    }
};

// The pair partition of one batch (or sub-round) into set `set` of own.
template <int KB, bool G>
template <class SR, class RM>
void MergeRun<KB, G>::launch_pairs(uint32_t cnt, const SR& sr, const RM& rm, const OwnerGeom& og, uint32_t set,
                                   uint32_t pset, hipStream_t st, Profiler* prof, hipEvent_t before_scatter) const {
    const unsigned tiles = pair_tiles_max(cnt);
    Timed tm(prof, st, SF_K_PAIRS, cnt);
    k_pair_count<KB, G, SR, RM><<<dim3(tiles, og.d), kCountThreads, 0, st>>>(meta, ent_key, cap, sr, rm, og,
                                                                            own->hmat);
    k_pair_colscan<><<<blocks_for(og.ncol, kScanCols), kScanCols * kScanWaves, 0, st>>>(own->hmat, meta,
                                                                                      own->pm[pset], og.ncol);
    k_pair_start<><<<1, 1024, 0, st>>>(own->pm[pset], og.ncol, meta, side_atomic ? 0u : 1u);
    if (before_scatter) own->mark(hipStreamWaitEvent(st, before_scatter, 0));
    k_pair_scatter<KB, G, SR, RM><<<dim3(tiles, og.d), kPairThreads, 0, st>>>(
        meta, ent_key, ent_cnt, cap, sr, rm, og, own->hmat, own->pm[pset], own->pairs[set], own->pos, cap);
}

template <int KB, bool G>
template <int D, class SR>
void MergeRun<KB, G>::launch_owner(uint32_t cnt, const SR& sr, bool ins, bool del, hipStream_t st, hipStream_t ps,
                                   Profiler* prof) const {
    const unsigned tiles = pair_tiles_max(cnt);
    if constexpr (!G) {
        // lone sketch: this batch's S1 + S2 share one owner step with the
        // previous batch's S3..S5; its own S3..S5 wait for the next step.  The
        // pairs come from ps; their scatter overwrites pairs and pos of two
        // batches back, which the previous batch's step and k_level read.
        const OwnerGeom& og = own->og;
        const uint32_t set = own->cur, prev = set ^ 1u;
        const uint32_t pset = own->pmc, pprev = (own->pmc + 2u) % 3u;
        const bool two = ps != st;
        launch_pairs(cnt, sr, LoneRanges{}, og, set, pset, ps, prof, two && own->l_rec ? own->ev_l : nullptr);
        if (two) {
            own->mark(hipEventRecord(own->ev_p, ps));
            own->mark(hipStreamWaitEvent(st, own->ev_p, 0));
        }
        {
            Timed tm(prof, st, SF_K_OWN_STEP, cnt);
            launch_own_step(og.d * og.R, own_step_lds(sr.g, og), st, sr, LoneRanges{}, og,
                            own->pending ? own->pm[pprev] : nullptr, own->pending ? own->pairs[prev] : nullptr,
                            own->level, ins ? own->pm[pset] : nullptr, ins ? own->pairs[set] : nullptr, own->res);
        }
        if (ins && !two && !(prof && prof->on)) {
            // one stream: T of this batch is taken in the next batch's first launch
            // (or alone when the call or the path ends there)
            own->level_due = true;
            own->level_pset = pset;
            own->level_tiles = tiles;
            own->level_keys = ent_key;
            own->level_flush = &flush_level<D, KB>;
        } else if (ins) {
            Timed tm(prof, st, SF_K_LEVEL, cnt);
            k_level<D><<<tiles, kPairThreads, 0, st>>>(own->pm[pset], ent_key, LoneRanges{}, own->pos, cap,
                                                       own->res, og.d, own->level);
        }
        if (two) {
            own->mark(hipEventRecord(own->ev_l, st));
            own->l_rec = true;
        }
        own->pending = true;  // this batch's S3..S5 (raise, deletes, clamp) come next
        own->cur = prev;
        own->pmc = (own->pmc + 1u) % 3u;
    } else {
        // sketch table: every sub-round is finished at once (the next one holds
        // other sketches): pairs, S1 + S2, T, then S3..S5
        const OwnerGeom og = sub_og;
        launch_pairs(cnt, sr, sub_rm, og, 0u, 0u, st, prof);
        const size_t lds = size_t(1) << og.cr_shift;
        const size_t lds_bytes = lds * (max_z + 1) * 4;
        if (ins) {
            {
                Timed tm(prof, st, SF_K_OWN_STEP, cnt);
                launch_own_step(og.d * og.R, lds_bytes, st, sr, sub_rm, og, nullptr, nullptr, own->level, own->pm[0],
                                own->pairs[0], own->res);
            }
            Timed tm(prof, st, SF_K_LEVEL, cnt);
            k_level<D><<<tiles, kPairThreads, 0, st>>>(own->pm[0], ent_key, sub_rm, own->pos, cap, own->res,
                                                       og.d, own->level);
        }
        Timed tm(prof, st, SF_K_OWN_FINAL, cnt);
        launch_own_step(og.d * og.R, lds_bytes, st, sr, sub_rm, og, own->pm[0], own->pairs[0], own->level, nullptr,
                        nullptr, own->res);
    }
    (void)del;
    (void)ps;
}

template <template <int> class PT>
struct Steps {
    template <int KB, int D>
    static void by_tile(uint32_t j, const PT<KB>& plan, unsigned tiles, bool ins, bool del, uint32_t* bpre,
                        uint16_t* asnap, uint32_t stride, hipStream_t st, Profiler* prof, uint64_t items) {
        switch (j) {
            case 1: launch_steps<KB, D, 1>(plan, tiles, ins, del, bpre, asnap, stride, st, prof, items); break;
            case 4: launch_steps<KB, D, 4>(plan, tiles, ins, del, bpre, asnap, stride, st, prof, items); break;
            default: launch_steps<KB, D, 8>(plan, tiles, ins, del, bpre, asnap, stride, st, prof, items); break;
        }
    }
    template <int KB>
    static void by_rows(uint32_t d, uint32_t j, const PT<KB>& plan, unsigned tiles, bool ins, bool del,
                        uint32_t* bpre, uint16_t* asnap, uint32_t stride, hipStream_t st, Profiler* prof,
                        uint64_t items) {
        if (d == 4) by_tile<KB, 4>(j, plan, tiles, ins, del, bpre, asnap, stride, st, prof, items);
        else if (d == 8) by_tile<KB, 8>(j, plan, tiles, ins, del, bpre, asnap, stride, st, prof, items);
        else by_tile<KB, 0>(j, plan, tiles, ins, del, bpre, asnap, stride, st, prof, items);
    }
};

template <int KB, class P, typename S>
void launch_query_rows(uint32_t d, const P& plan, unsigned tiles, hipStream_t st) {
    const dim3 grid(tiles), block(kBlock);
    if (d == 4) k_query<KB, 4, S, P><<<grid, block, 0, st>>>(plan);
    else if (d == 8) k_query<KB, 8, S, P><<<grid, block, 0, st>>>(plan);
    else k_query<KB, 0, S, P><<<grid, block, 0, st>>>(plan);
}

}  // namespace sfh
