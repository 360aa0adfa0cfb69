// SF-sketch kernels (gfx950).  Every kernel takes a work plan that tells each
// workgroup which tile of ops (or query keys) it owns and in which sketch:
//   UniformPlan  one sketch, one schedule batch, tile = blockIdx (no table)
//   ListPlan     a device table of tiles over many sketches (sketch groups)
// The step each kernel implements is the same in both cases.
//
// One schedule batch (the sf.h update schedule), S1..S5:
//   S1  insert keys: Slim and Fat counters before the batch
//   S2  insert keys: Fat += count
//   S3  insert keys: T = min(m0 + delta, max(m0, Bmin), 65535), atomic max
//       into the Slim where T exceeds it
//   S4  delete keys: Fat -= count
//   S5  delete keys: atomic min of the Slim with the bucket max
// Two ways to get there, with identical results:
//   batch-wide merging (default): k_part_count / k_part_colscan /
//     k_part_start / k_part_scatter partition the batch's keys into hash
//     buckets, k_merge turns each bucket chunk into entries (key, count), and
//     k_entries_snapshot / _fat / _raise / _fat / _clamp run S1..S5 once per
//     entry;
//   per-tile merging: k_snapshot, k_fat_update, k_raise, k_fat_update,
//     k_clamp each group the duplicate keys of their tile in LDS first.
// Kernel boundaries are the schedule's grid-wide barriers.  A cell of the
// sketch is one record of z+1 uint32 words: its Fat bucket, then its Slim
// working copy (Geom::rs words apart from the next cell's).
#pragma once

#include "sf_device.hpp"

namespace sfk {

// How the ops of a tile are typed.
enum OpMode : uint32_t { kOpsArray = 0, kAllInsert = 1, kAllDelete = 2 };

// What one workgroup processes.
struct Work {
    const uint8_t* keys;  // first key of the tile
    const uint8_t* ops;   // first op code of the tile (kOpsArray only)
    uint32_t* out;        // first query answer of the tile (queries only)
    uint32_t count;       // ops (or query keys) in the tile
    uint32_t scr;         // snapshot index of the tile's first op
    uint32_t mode;        // OpMode
    uint32_t sketch;      // index of the tile's sketch in its table (0 for a lone sketch)
    Geom g;
    uint32_t* fat;
    void* slim;           // uint32 working copy (updates) or uint16 export (collector queries)
};

template <int KB> struct UniformPlan {
    const uint8_t* keys;
    const uint8_t* ops;
    uint32_t* out;
    uint32_t cnt;
    uint32_t mode;
    Geom g;
    uint32_t* fat;
    void* slim;
    __device__ __forceinline__ Work at(uint32_t blk, uint32_t tile_ops) const {
        const uint32_t first = blk * tile_ops;
        const uint32_t rest = cnt - first;
        return Work{keys + size_t(first) * KB, ops ? ops + first : nullptr, out ? out + first : nullptr,
                    rest < tile_ops ? rest : tile_ops, first, mode, 0u, g, fat, slim};
    }
};

struct TileDesc {         // one tile of a ListPlan
    const uint8_t* keys;  // its first key
    const uint8_t* ops;   // its first op code (kOpsArray), else null
    uint32_t* out;        // its first answer (queries), else null
    uint32_t count;       // ops or keys in the tile
    uint32_t sketch;      // index into the sketch table
    uint32_t scr;         // snapshot index of its first op (within the launch round)
    uint32_t mode;        // OpMode
};

struct SketchDesc {       // one sketch of a group or pool
    Geom g;
    uint32_t* fat;
    uint32_t* slim;
};

template <int KB> struct ListPlan {
    const TileDesc* tiles;
    const SketchDesc* sketches;
    __device__ __forceinline__ Work at(uint32_t blk, uint32_t) const {
        const TileDesc t = tiles[blk];
        const SketchDesc s = sketches[t.sketch];
        return Work{t.keys, t.ops, t.out, t.count, t.scr, t.mode, t.sketch, s.g, s.fat, s.slim};
    }
};

__device__ __forceinline__ bool is_delete(const uint8_t* ops, uint32_t t, uint32_t mode) {
    return mode == kOpsArray ? ops[t] != 0 : mode == kAllDelete;
}

#define SF_ROWS(D, g) (D ? uint32_t(D) : (g).d)

// S1: snapshot of each insert op's Slim and Fat counters (state before the batch).
template <int KB, int D, int J, class P>
__global__ __launch_bounds__(kBlock) void k_snapshot(P plan, uint32_t* __restrict__ bpre,
                                                     uint16_t* __restrict__ asnap, uint32_t stride) {
    const Work w = plan.at(blockIdx.x, kBlock * J);
    const uint32_t* slim = static_cast<const uint32_t*>(w.slim);
    const uint32_t d = SF_ROWS(D, w.g);
#pragma unroll
    for (int j = 0; j < J; j++) {
        const uint32_t t = uint32_t(j) * kBlock + threadIdx.x;
        if (t >= w.count || is_delete(w.ops, t, w.mode)) continue;
        const Mixed<KB> mx(load_key<KB>(w.keys, t));
        const size_t s = size_t(w.scr) + t;
#pragma unroll
        for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
            if (i < d) {
                uint32_t h, f;
                split(w.g, mx.row(w.g.seed_base + i), h, f);
                const size_t cell = size_t(i) * w.g.w + h;
                asnap[size_t(i) * stride + s] = uint16_t(slim[cell * w.g.rs]);
                bpre[size_t(i) * stride + s] = w.fat[cell * w.g.rs + f];
            }
        }
    }
}

// Loads the tile's active ops (op type == want_del) into the LDS table.
// Returns after a barrier; the table then holds each distinct key once.
template <int KB, int J>
__device__ __forceinline__ void tile_build(TileLDS<KB, J>& L, const Work& w, bool want_del) {
    tile_clear<KB, J>(L);
    Key<KB> k[J];
    bool act[J];
#pragma unroll
    for (int j = 0; j < J; j++) {
        const uint32_t idx = uint32_t(j) * kBlock + threadIdx.x;
        act[j] = idx < w.count && is_delete(w.ops, idx, w.mode) == want_del;
        if (act[j]) {
            k[j] = load_key<KB>(w.keys, idx);
            L.key[idx] = k[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; j++)
        if (act[j]) tile_insert<KB, J>(L, k[j], uint32_t(j) * kBlock + threadIdx.x);
    __syncthreads();
}

// S2 / S4: Fat counters of every insert (want_del = 0) or delete (want_del = 1)
// op move by one: one atomic per distinct key of the tile, carrying its count.
template <int KB, int D, int J, class P>
__global__ __launch_bounds__(kBlock) void k_fat_update(P plan, uint32_t want_del) {
    __shared__ TileLDS<KB, J> L;
    const Work w = plan.at(blockIdx.x, kBlock * J);
    tile_build<KB, J>(L, w, want_del != 0);
    const uint32_t d = SF_ROWS(D, w.g);
    for (uint32_t s = threadIdx.x; s < TileLDS<KB, J>::kSlots; s += kBlock) {
        const uint32_t o = L.owner[s];
        if (o == kEmpty) continue;
        const uint32_t n = L.cnt[s];
        const uint32_t v = want_del ? 0u - n : n;
        const Mixed<KB> mx(L.key[o]);
#pragma unroll
        for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
            if (i < d) {
                uint32_t h, f;
                split(w.g, mx.row(w.g.seed_base + i), h, f);
                atomic_add_u32(&w.fat[(size_t(i) * w.g.w + h) * w.g.rs + f], v);
            }
        }
    }
}

// S3: raise the Slim counters of every inserted key to its water level
// T = min(m0 + delta, max(m0, Bmin), 65535), once per distinct key of the tile.
template <int KB, int D, int J, class P>
__global__ __launch_bounds__(kBlock) void k_raise(P plan, const uint32_t* __restrict__ bpre,
                                                  const uint16_t* __restrict__ asnap, uint32_t stride) {
    constexpr int R = D ? D : kMaxD;
    __shared__ TileLDS<KB, J> L;
    const Work w = plan.at(blockIdx.x, kBlock * J);
    tile_build<KB, J>(L, w, false);
    uint32_t* slim = static_cast<uint32_t*>(w.slim);
    const uint32_t d = SF_ROWS(D, w.g);
    for (uint32_t s = threadIdx.x; s < TileLDS<KB, J>::kSlots; s += kBlock) {
        const uint32_t o = L.owner[s];
        if (o == kEmpty) continue;
        const size_t t = size_t(w.scr) + o;  // any op of the key: all share one snapshot
        const Mixed<KB> mx(L.key[o]);
        size_t cell[R];
        uint32_t a[R];
        uint32_t m0 = ~0u, bmin = ~0u, delta = ~0u;
#pragma unroll
        for (int i = 0; i < R; i++) {
            cell[i] = 0;
            a[i] = kSlimMax;
            if (uint32_t(i) < d) {
                uint32_t h, f;
                split(w.g, mx.row(w.g.seed_base + i), h, f);
                cell[i] = size_t(i) * w.g.w + h;
                a[i] = asnap[size_t(i) * stride + t];
                const uint32_t post = w.fat[cell[i] * w.g.rs + f];
                const uint32_t grew = post - bpre[size_t(i) * stride + t];
                m0 = min(m0, a[i]);
                bmin = min(bmin, post);
                delta = min(delta, grew);
            }
        }
        const uint64_t rise = uint64_t(m0) + delta;
        const uint64_t level = m0 > bmin ? m0 : bmin;
        const uint64_t tt = rise < level ? rise : level;
        const uint32_t T = uint32_t(tt < kSlimMax ? tt : kSlimMax);
#pragma unroll
        for (int i = 0; i < R; i++)
            if (uint32_t(i) < d && a[i] < T) atomic_max_u32(&slim[cell[i] * w.g.rs], T);
    }
}

// Largest counter of a Fat bucket (the first z words of the cell's record).
__device__ __forceinline__ uint32_t bucket_max(const uint32_t* __restrict__ fat, size_t cell,
                                               const Geom& g) {
    const uint32_t* b = fat + cell * g.rs;
    if (g.z == 4) return max(max(b[0], b[1]), max(b[2], b[3]));
    uint32_t m = 0;
    for (uint32_t j = 0; j < g.z; j++) m = max(m, b[j]);
    return m;
}

// S5: clamp the Slim counters of every deleted key to their bucket's max,
// once per distinct key of the tile.
template <int KB, int D, int J, class P>
__global__ __launch_bounds__(kBlock) void k_clamp(P plan) {
    __shared__ TileLDS<KB, J> L;
    const Work w = plan.at(blockIdx.x, kBlock * J);
    tile_build<KB, J>(L, w, true);
    uint32_t* slim = static_cast<uint32_t*>(w.slim);
    const uint32_t d = SF_ROWS(D, w.g);
    for (uint32_t s = threadIdx.x; s < TileLDS<KB, J>::kSlots; s += kBlock) {
        const uint32_t o = L.owner[s];
        if (o == kEmpty) continue;
        const Mixed<KB> mx(L.key[o]);
#pragma unroll
        for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
            if (i < d) {
                uint32_t h, f;
                split(w.g, mx.row(w.g.seed_base + i), h, f);
                const size_t cell = size_t(i) * w.g.w + h;
                const uint32_t m = bucket_max(w.fat, cell, w.g);
                if (slim[cell * w.g.rs] > m) atomic_min_u32(&slim[cell * w.g.rs], m);
            }
        }
    }
}

// Point query: minimum of the d Slim counters of each key (one key per lane).
template <int KB, int D, typename S, class P>
__global__ __launch_bounds__(kBlock) void k_query(P plan) {
    const Work w = plan.at(blockIdx.x, kBlock);
    const uint32_t t = threadIdx.x;
    if (t >= w.count) return;
    const S* slim = static_cast<const S*>(w.slim);
    // a uint32 Slim is the working copy inside the cell records; a uint16 one
    // is a dense exported [d][w] array
    const uint32_t qs = sizeof(S) == 4 ? w.g.rs : 1u;
    const Mixed<KB> mx(load_key<KB>(w.keys, t));
    const uint32_t d = SF_ROWS(D, w.g);
    uint32_t q = ~0u;
#pragma unroll
    for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
        if (i < d) {
            uint32_t h, f;
            split(w.g, mx.row(w.g.seed_base + i), h, f);
            q = min(q, uint32_t(slim[(size_t(i) * w.g.w + h) * qs]));
        }
    }
    w.out[t] = q;
}

// The Fat-subsketch in its dense [d][w][z] form, out of the cell records.
// Point query over a dense uint16 Slim [d][w], one row per XCD.  The
// dispatcher deals workgroups to the 8 XCDs round-robin, so workgroup b runs
// on XCD b % 8.  With d dividing 8, XCD x reads only row x % d (2 MiB at
// w = 2^20, which its 4 MB L2 holds) and takes every (8/d)-th run of kBlock
// keys.  part[r][t] receives row r's counter of key t; k_query_min takes the
// minimum over the rows.  Placement only decides cache hits: any other
// dispatch order gives the same answers.  gridDim.x is a multiple of 8.
constexpr uint32_t kXcds = 8;
template <int KB>
__global__ __launch_bounds__(kBlock) void k_query_rows(const uint8_t* __restrict__ keys, uint32_t n,
                                                       const uint16_t* __restrict__ view, Geom g, uint32_t d,
                                                       uint16_t* __restrict__ part) {
    const uint32_t x = blockIdx.x % kXcds, r = x % d, nsub = kXcds / d;
    const uint32_t slot = (blockIdx.x / kXcds) * nsub + x / d, nslots = (gridDim.x / kXcds) * nsub;
    const uint16_t* row = view + size_t(r) * g.w;
    for (uint32_t t = slot * kBlock + threadIdx.x; t < n; t += nslots * kBlock) {
        uint32_t h, f;
        split(g, Mixed<KB>(load_key<KB>(keys, t)).row(g.seed_base + r), h, f);
        part[size_t(r) * n + t] = row[h];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_query_min(const T* __restrict__ part, uint32_t n, uint32_t d,
                                                      uint32_t* __restrict__ out) {
    for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < n; t += gridDim.x * kBlock) {
        uint32_t m = part[t];
        for (uint32_t r = 1; r < d; r++) m = min(m, uint32_t(part[size_t(r) * n + t]));
        out[t] = m;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_unpack_fat(const T* __restrict__ rec, T* __restrict__ out,
                                                       size_t cells, uint32_t z) {
    const size_t n = cells * z;
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock)
        out[i] = rec[(i / z) * (z + 1) + i % z];
}

// Narrowing copy of a 32-bit Slim working copy (every stride-th word) into
// the dense uint16 export form (to out, and to out2 unless it is null).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack16(const T* __restrict__ in, uint16_t* __restrict__ out,
                                                   size_t n, uint32_t stride, uint16_t* __restrict__ out2) {
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock) {
        const uint16_t v = uint16_t(in[i * stride]);
        out[i] = v;
        if (out2) out2[i] = v;
    }
}

}  // namespace sfk

// =====================================================================
// Batch-wide duplicate merging ("batch merge").  The tile kernels above
// merge duplicates inside each tile only; on skewed streams most of a
// batch's ops repeat keys seen in other tiles.  Here the batch's keys are
// first partitioned into nb hash buckets per op type, then one workgroup per
// chunk of a bucket merges them in an LDS table, emitting one entry (key,
// count) per distinct key of the chunk.  Insert entries grow up from index
// 0, delete entries down from the last index, so both fit the snapshot
// scratch of one batch.  S1..S5 then run once per entry.  In sketch groups
// and pools the merged key carries its sketch's index (G = true) and every
// entry kernel looks its sketch up in the table.
// =====================================================================
namespace sfk {

constexpr uint32_t kMaxBuckets = 1024;         // per op type; the runtime nb is a power of two <= this
constexpr uint32_t kPartOps = 8192;            // ops per partitioning workgroup
constexpr uint32_t kPartOpsWide = 16384;       // ... for a lone sketch's large batches of uint32 keys
constexpr uint32_t kWideBatch = 1u << 22;      // (batches of at least this many ops)
constexpr uint32_t kPartThreads = 1024;        // its threads (16 waves)
// Partitioning groups one batch (or merged sub-round) of cap ops may use:
// full tiles plus one partial tile per sketch, at most extra sketches.
__host__ __device__ constexpr uint64_t part_groups_max(uint64_t cap, uint64_t extra) {
    return (cap + kPartOps - 1) / kPartOps + extra;
}

template <int KB, bool G> struct MKey { Key<KB> k; };
template <int KB> struct MKey<KB, true> { Key<KB> k; uint32_t s; };

template <int KB, bool G>
__device__ __forceinline__ MKey<KB, G> mkey(const Key<KB>& k, uint32_t sketch) {
    MKey<KB, G> m;
    m.k = k;
    if constexpr (G) m.s = sketch;
    return m;
}
template <int KB, bool G> __device__ __forceinline__ uint32_t mkey_sketch(const MKey<KB, G>& m) {
    if constexpr (G) return m.s;
    else return 0u;
}
template <int KB, bool G> __device__ __forceinline__ bool mkey_eq(const MKey<KB, G>& a, const MKey<KB, G>& b) {
    if constexpr (G) return a.s == b.s && key_eq<KB>(a.k, b.k);
    else return key_eq<KB>(a.k, b.k);
}
template <int KB, bool G> __device__ __forceinline__ uint32_t mkey_hash(const MKey<KB, G>& m) {
    if constexpr (G) {
        uint32_t h = 0x9e3779b9u;
#pragma unroll
        for (int j = 0; j < int(sizeof(m.k.v) / 4); j++) h = mm_round(h, mm_mix(m.k.v[j]));
        return mm_final(mm_round(h, mm_mix(m.s)), 0u);
    } else {
        return slot_hash<KB>(m.k);
    }
}

template <int KB, bool G> struct MergeShape {  // LDS table of the merging kernel
    // uint32 keys: chunks of 8192 keys and 12280 slots for a lone sketch,
    // 6144 (key, sketch) pairs and 8190 slots in groups and pools -- either
    // way keys and slots take just under 80 KB, so two groups of 16 waves
    // share a CU.  13-byte keys: 2048 per chunk, 4096 slots (8 waves).
    static constexpr uint32_t kThreads = KB == 4 ? 1024 : 512;
    static constexpr int J = KB == 4 ? (G ? 6 : 8) : 4;
    static constexpr uint32_t kChunk = kThreads * J;
    static constexpr uint32_t kSlots = KB == 4 ? (G ? 8190u : 12280u) : 2 * kChunk;
    static_assert(kSlots > kChunk, "a chunk's keys always fit the table");
};
constexpr uint32_t kMinChunk = 2048;  // smallest kChunk of any shape

// One merge chunk: a range of the partitioned keys, and the buckets
// [b_lo, b_hi) it holds whole (empty for a piece of a split bucket).
struct MergeChunk {
    uint32_t first, n, del, b_lo, b_hi;
};
// An insert entry whose row-0 S1 and S2 the merge took in place carries this
// bit in its count (counts stay below 2^16).
constexpr uint32_t kRow0Done = 0x80000000u;
// Chunks one batch (or merged sub-round) of cap ops can have: full chunks
// plus one partial chunk per bucket.
__host__ __device__ constexpr uint64_t merge_chunks_max(uint64_t cap) { return cap / kMinChunk + 2 * kMaxBuckets + 1; }

// Bucket count for a batch of cnt ops: about one chunk of ops per bucket, so
// that few keys are split between two chunks (each part becomes an entry).  A
// sketch table stops at half the limit: there a batch holds many sketches'
// short per-sketch batches, whose duplicates already meet in a bucket of two
// or three chunks, and the wider histogram matrix would cost more than it
// saves.
template <int KB, bool G> __host__ __device__ inline uint32_t buckets_for(uint64_t cnt) {
    constexpr uint32_t kLimit = G ? kMaxBuckets / 2 : kMaxBuckets;
    uint32_t nb = 16;
    while (nb < kLimit && uint64_t(nb) * MergeShape<KB, G>::kChunk < cnt) nb <<= 1;
    return nb;
}

// The merge table packs a slot's owner (local key index) and count into one
// word -- owner in the high half, count in the low half.
template <int KB, bool G> struct MergeLDS {
    MKey<KB, G> key[MergeShape<KB, G>::kChunk];
    uint32_t slot[MergeShape<KB, G>::kSlots];
};

// Adds cnt copies of key k (local index idx) to the first `slots` slots of
// the table.  Returns the slot if this call created it (the key was new),
// else kEmpty.
template <int KB, bool G>
__device__ __forceinline__ uint32_t merge_insert(MergeLDS<KB, G>& L, const MKey<KB, G>& k, uint32_t idx,
                                                 uint32_t cnt, uint32_t slots) {
    const uint32_t h = mkey_hash<KB, G>(k);
    // a sketch table's bucket came from the hash's top bits, so the slot
    // starts from the low ones
    uint32_t s = __umulhi(__builtin_rotateleft32(h, 16), slots);
    for (uint32_t probe = 0; probe < slots; probe++) {
        const uint32_t prev = atomicCAS(&L.slot[s], kEmpty, (idx << 16) | cnt);
        if (prev == kEmpty) return s;
        if (mkey_eq<KB, G>(L.key[prev >> 16], k)) {
            atomicAdd(&L.slot[s], cnt);  // counts stay < 2^16: never carry into the owner
            return kEmpty;
        }
        s = s + 1 == slots ? 0u : s + 1;
    }
    return kEmpty;
}

// Value of x in lane `lane` (wave-uniform) of the wavefront.
template <class T> __device__ __forceinline__ T read_lane(const T& x, int lane) {
    static_assert(sizeof(T) % 4 == 0, "read_lane moves whole dwords");
    T r;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&x);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); i++) dst[i] = __builtin_amdgcn_readlane(src[i], lane);
    return r;
}

// Skewed streams put many copies of one key in one wavefront, and LDS
// atomics on one address serialise.  K rounds of "peeling": the first
// unclaimed lane leads, every lane holding the leader's value joins it, and
// the leader alone carries the group.  Returns this lane's weight: the group
// size for a leader, 0 for a follower (or an invalid lane), 1 for a lane left
// unclaimed.  Call with the whole wavefront.
template <int K, class T, class Eq>
__device__ __forceinline__ uint32_t wave_peel(const T& v, bool valid, Eq eq) {
    bool claimed = !valid;
    uint32_t w = valid ? 1u : 0u;
    const int lane = int(lane_id());
#pragma unroll
    for (int r = 0; r < K; r++) {
        const unsigned long long act = __ballot(!claimed);
        if (act == 0) break;
        const int leader = __ffsll(act) - 1;
        const T lv = read_lane(v, leader);
        const bool same = !claimed && eq(v, lv);
        const unsigned long long m = __ballot(same);
        if (same) {
            claimed = true;
            w = lane == leader ? uint32_t(__popcll(m)) : 0u;
        }
    }
    return w;
}

constexpr int kPeel = 2;

struct MergeMeta {                    // device-side bookkeeping of one batch
    uint32_t total[2 * kMaxBuckets];  // keys per bucket (written by k_part_colscan)
    uint32_t start[2 * kMaxBuckets];  // first position of each bucket in the partitioned keys
    uint32_t size[2 * kMaxBuckets];
    uint32_t chunk0[2 * kMaxBuckets + 1];  // chunks of the buckets before each bucket (prefix; [nbt] = all)
    // Entries emitted.  Every merging workgroup bumps one of these once, so
    // each sits on its own 256-byte line (atomics on one line serialise).
    alignas(256) uint32_t n_ins;
    alignas(256) uint32_t n_del;
    alignas(256) unsigned long long acc_ins;  // entries emitted since creation
    unsigned long long acc_del;
};

// The partition takes no global atomics: each group writes its bucket
// histogram to its row of hist [groups][nbt]; k_part_colscan turns every
// column into the groups' offsets inside the bucket (and the bucket total);
// k_part_start lays the buckets out; k_part_scatter adds the two.

// Bucket of a key.  A lone sketch buckets by the key's row-0 cell (nb equal
// cell ranges), so the entries one merge chunk emits -- processed side by
// side by the entry kernels -- share a narrow range of row-0 cell records
// that stays in cache.  With a sketch table it is the top log2(nb) bits of
// the key's hash.  (The merge table's slot comes from a different hash.)
// floor(h * 2^nb_log2 / w) for widths that are no power of two, kept out of
// line: a 64-bit division inlined once per key bloats the partition kernels.
__device__ __noinline__ uint32_t bucket_div(uint32_t h, uint32_t nb_log2, uint32_t w) {
    return uint32_t((uint64_t(h) << nb_log2) / w);
}

template <int KB, bool G>
__device__ __forceinline__ uint32_t bucket_of(const MKey<KB, G>& k, bool del, uint32_t nb_log2, const Geom& g) {
    uint32_t b;
    if constexpr (G) {
        b = mkey_hash<KB, G>(k) >> (32u - nb_log2);
    } else {
        uint32_t h, f;
        split(g, Mixed<KB>(k.k).row(g.seed_base), h, f);
        if (g.pow2)  // floor(h * nb / w) with both powers of two
            b = g.w_shift >= nb_log2 ? h >> (g.w_shift - nb_log2) : h << (nb_log2 - g.w_shift);
        else
            b = bucket_div(h, nb_log2, g.w);
    }
    return b + (del ? (1u << nb_log2) : 0u);
}

// Inclusive scan under op over the workgroup's threads in thread order
// (blockDim.x <= 1024): a shuffle scan inside each wavefront, then one over
// the wavefront totals.  tmp: 16 words of LDS.  Call with the whole workgroup.
template <class Op>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, Op op, uint32_t identity, uint32_t* tmp) {
    const uint32_t lane = lane_id(), wv = threadIdx.x / 64, nw = (blockDim.x + 63) / 64;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t x = __shfl_up(v, off);
        if (lane >= uint32_t(off)) v = op(v, x);
    }
    if (lane == 63u || threadIdx.x == blockDim.x - 1) tmp[wv] = v;  // the wavefront's total
    __syncthreads();
    if (wv == 0) {
        uint32_t t = lane < nw ? tmp[lane] : identity;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const uint32_t x = __shfl_up(t, off);
            if (lane >= uint32_t(off)) t = op(t, x);
        }
        if (lane < nw) tmp[lane] = t;
    }
    __syncthreads();
    v = wv ? op(tmp[wv - 1], v) : v;
    __syncthreads();  // tmp is free again
    return v;
}
struct AddOp {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};
struct MinOp {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a < b ? a : b; }
};

// Row of tile b (of n) in a histogram matrix, numbering the tiles XCD by XCD:
// the dispatcher deals workgroups to the 8 XCDs round-robin, so tile b runs
// on XCD b % 8, and with this order the runs that one XCD's tiles write into
// a bucket (or column) are contiguous: few lines of the partitioned output
// are written from two XCDs' L2s.  Any bijection gives the same results (the
// order inside a bucket is free); this one only decides the write traffic.
__device__ __forceinline__ uint32_t xcd_row(uint32_t b, uint32_t n) {
    const uint32_t x = b % 8u, q = n / 8u, r = n % 8u;
    return x * q + min(x, r) + b / 8u;
}

// The thread's R keys of a partition tile (kPartThreads apart) and their op
// types, every load issued before any is used: the loop bodies hold no
// branch, so they stay in one basic block.  Slots past the tile's end load
// its first key and must be skipped by the caller (t >= w.count).
template <int KB, bool G, uint32_t R>
__device__ __forceinline__ void load_tile_keys(const Work& w, MKey<KB, G> (&k)[R], bool (&del)[R]) {
    uint32_t opb[R];
    if (w.mode == kOpsArray) {
#pragma unroll
        for (uint32_t r = 0; r < R; r++) {
            const uint32_t t = r * kPartThreads + threadIdx.x;
            opb[r] = w.ops[t < w.count ? t : 0u];
        }
    } else {
#pragma unroll
        for (uint32_t r = 0; r < R; r++) opb[r] = w.mode == kAllDelete ? 1u : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < R; r++) {
        const uint32_t t = r * kPartThreads + threadIdx.x;
        k[r] = mkey<KB, G>(load_key<KB>(w.keys, t < w.count ? t : 0u), w.sketch);
    }
#pragma unroll
    for (uint32_t r = 0; r < R; r++) del[r] = opb[r] != 0;
}

// Counts the ops of every bucket in each group's tile.
// The histogram of tile blk (of ntiles): one workgroup of kPartThreads.
template <int KB, bool G, class P, uint32_t OPS>
__device__ __forceinline__ void part_count_tile(const P& plan, uint32_t* __restrict__ hist_out, uint32_t nb_log2,
                                                uint32_t blk, uint32_t ntiles) {
    constexpr uint32_t R = OPS / kPartThreads;  // keys per thread (a tile holds at most OPS)
    __shared__ uint32_t hist[2 * kMaxBuckets];
    const uint32_t nbt = 2u << nb_log2;
    const Work w = plan.at(blk, OPS);
    for (uint32_t b = threadIdx.x; b < nbt; b += kPartThreads) hist[b] = 0;
    MKey<KB, G> k[R];
    bool del[R];
    if (w.count) load_tile_keys<KB, G, R>(w, k, del);
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < R; r++) {
        if (r * kPartThreads + threadIdx.x < w.count) atomicAdd(&hist[bucket_of<KB, G>(k[r], del[r], nb_log2, w.g)], 1u);
    }
    __syncthreads();
    const uint32_t row = xcd_row(blk, ntiles);
    for (uint32_t b = threadIdx.x; b < nbt; b += kPartThreads) hist_out[size_t(row) * nbt + b] = hist[b];
}

template <int KB, bool G, class P, uint32_t OPS = kPartOps>
__global__ __launch_bounds__(kPartThreads) void k_part_count(P plan, uint32_t* __restrict__ hist_out,
                                                         uint32_t nb_log2) {
    part_count_tile<KB, G, P, OPS>(plan, hist_out, nb_log2, blockIdx.x, gridDim.x);
}

// Column scans of hist: 64 buckets per workgroup, one per lane, so that a
// wavefront reads 256 contiguous bytes of a row; the 16 wavefronts split the
// groups into segments.  hist[g][b] becomes the number of bucket-b keys of
// groups < g.  A segment of at most 64 rows stays in registers between the
// sum and the prefix pass; longer ones are read twice.
constexpr uint32_t kScanCols = 64, kScanWaves = 16, kScanRowsReg = 64;
template <typename T>
__device__ __forceinline__ void colscan_wide(T* __restrict__ hist, uint32_t groups, uint32_t nbt,
                                             uint32_t* __restrict__ totals) {
    __shared__ T seg_sum[kScanWaves][kScanCols];
    const uint32_t lane = lane_id(), wv = threadIdx.x / 64;
    const uint32_t b = blockIdx.x * kScanCols + lane;
    const uint32_t rows = (groups + kScanWaves - 1) / kScanWaves;
    const uint32_t g0 = wv * rows, g1 = min(groups, g0 + rows);
    const bool in_reg = rows <= kScanRowsReg;
    T v[kScanRowsReg];
    T sum = 0;
    if (b < nbt) {
        if (in_reg) {
#pragma unroll
            for (uint32_t r = 0; r < kScanRowsReg; r++) {
                v[r] = g0 + r < g1 ? hist[size_t(g0 + r) * nbt + b] : T(0);
                sum += v[r];
            }
        } else {
            for (uint32_t g = g0; g < g1; g++) sum += hist[size_t(g) * nbt + b];
        }
    }
    seg_sum[wv][lane] = sum;
    __syncthreads();
    if (wv == 0) {                                // exclusive prefix over the segments, per column
        T run = 0;
#pragma unroll
        for (uint32_t w = 0; w < kScanWaves; w++) {
            const T x = seg_sum[w][lane];
            seg_sum[w][lane] = run;
            run += x;
        }
        if (b < nbt) totals[b] = run;
    }
    __syncthreads();
    T run = seg_sum[wv][lane];                    // keys of this bucket in earlier segments
    if (b < nbt) {
        if (in_reg) {
#pragma unroll
            for (uint32_t r = 0; r < kScanRowsReg; r++) {
                if (g0 + r < g1) hist[size_t(g0 + r) * nbt + b] = run;
                run += v[r];
            }
        } else {
            for (uint32_t g = g0; g < g1; g++) {
                const T x = hist[size_t(g) * nbt + b];
                hist[size_t(g) * nbt + b] = run;
                run += x;
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kScanCols * kScanWaves) void k_part_colscan(
    T* __restrict__ hist, uint32_t groups, uint32_t nbt, MergeMeta* __restrict__ meta) {
    colscan_wide<T>(hist, groups, nbt, meta->total);
}

// The same for other shapes -- a tall matrix (more than kScanWaves *
// kScanRowsReg groups, as in sketch groups and pools) or a short one (a small
// batch): 4 buckets per workgroup and the groups split into 64 segments, so
// that many workgroups share the rows.
constexpr uint32_t kScanBuckets = 4, kScanSegs = 64;
template <typename T>
__device__ __forceinline__ void colscan_tall(T* __restrict__ hist, uint32_t groups, uint32_t nbt,
                                             uint32_t* __restrict__ totals) {
    constexpr uint32_t kRowsReg = 16;             // a segment's rows kept in registers when it has few
    __shared__ T seg_sum[kScanSegs][kScanBuckets];
    const uint32_t lb = threadIdx.x % kScanBuckets, sg = threadIdx.x / kScanBuckets;
    const uint32_t b = blockIdx.x * kScanBuckets + lb;
    const uint32_t rows = (groups + kScanSegs - 1) / kScanSegs;
    const uint32_t g0 = sg * rows, g1 = min(groups, g0 + rows);
    const bool in_reg = rows <= kRowsReg;
    T v[kRowsReg];
    T sum = 0;
    if (b < nbt) {
        if (in_reg) {
#pragma unroll
            for (uint32_t r = 0; r < kRowsReg; r++) {
                v[r] = g0 + r < g1 ? hist[size_t(g0 + r) * nbt + b] : T(0);
                sum += v[r];
            }
        } else {
            for (uint32_t g = g0; g < g1; g++) sum += hist[size_t(g) * nbt + b];
        }
    }
    seg_sum[sg][lb] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < kScanSegs; off <<= 1) {  // inclusive scan over the segments
        const T x = sg >= off ? seg_sum[sg - off][lb] : T(0);
        __syncthreads();
        seg_sum[sg][lb] += x;
        __syncthreads();
    }
    T run = seg_sum[sg][lb] - sum;                // keys of this bucket in earlier segments
    if (b < nbt) {
        if (in_reg) {
#pragma unroll
            for (uint32_t r = 0; r < kRowsReg; r++) {
                if (g0 + r < g1) hist[size_t(g0 + r) * nbt + b] = run;
                run += v[r];
            }
        } else {
            for (uint32_t g = g0; g < g1; g++) {
                const T x = hist[size_t(g) * nbt + b];
                hist[size_t(g) * nbt + b] = run;
                run += x;
            }
        }
        if (sg == kScanSegs - 1) totals[b] = run;
    }
}
template <typename T>
__global__ __launch_bounds__(kScanBuckets * kScanSegs) void k_part_colscan_tall(
    T* __restrict__ hist, uint32_t groups, uint32_t nbt, MergeMeta* __restrict__ meta) {
    colscan_tall<T>(hist, groups, nbt, meta->total);
}

// One workgroup of nbt/2 threads (thread t owns buckets 2t and 2t+1): bucket
// starts, then the merge chunks, then clears the entry counters for the next
// batch.  A bucket of more than half a chunk of keys gets ceil(size / chunk)
// chunks of its own.  Smaller buckets are packed: consecutive small buckets
// of one op type whose starts fall in the same half-chunk window of the
// partitioned keys share one chunk.  Such a chunk spans less than half a
// chunk of starts plus a last bucket of at most half a chunk, so never more
// than a chunk.  Equal keys share a bucket, so packing never splits a key's
// copies between chunks.
constexpr uint32_t kStartPer = 2;
constexpr uint32_t kBigChunks = 8, kBigList = 64;
static_assert(2 * kMaxBuckets / kStartPer <= 1024, "k_part_start is one workgroup");
static_assert((2 * kMaxBuckets) % kPartThreads == 0, "k_part_scatter gives each thread whole buckets");
// The bucket layout of one batch, one workgroup of nbt / 2 threads.
template <int KB, bool G>
__device__ __forceinline__ void part_start_block(MergeMeta* __restrict__ meta, MergeChunk* __restrict__ chunks) {
    constexpr uint32_t K = MergeShape<KB, G>::kChunk, H = K / 2, P = kStartPer;
    static_assert(P == 2, "the group-end lookup below assumes two buckets per thread");
    __shared__ uint32_t tmp[16];
    __shared__ uint32_t rev[2 * kMaxBuckets / P];  // per-thread values in reverse thread order
    __shared__ uint32_t st[2 * kMaxBuckets + 1];   // bucket starts, then the end of the keys
    __shared__ uint32_t big_b[kBigList], big_c0[kBigList], nbig;  // buckets of more than kBigChunks chunks
    const uint32_t t = threadIdx.x, nt = blockDim.x, nbt = P * nt, half = nbt / 2;
    uint32_t sz[P], sum = 0;
#pragma unroll
    for (uint32_t e = 0; e < P; e++) {
        sz[e] = meta->total[t * P + e];
        sum += sz[e];
    }
    // bucket starts
    uint32_t first = block_scan(sum, AddOp{}, 0u, tmp) - sum;
#pragma unroll
    for (uint32_t e = 0; e < P; e++) {
        const uint32_t b = t * P + e;
        st[b] = first;
        meta->size[b] = sz[e];
        meta->start[b] = first;
        first += sz[e];
    }
    if (t == nt - 1) st[nbt] = first;
    __syncthreads();
    // where packed groups start: op type boundary, next to a big bucket, new window
    bool gs[P];
    uint32_t lo = nbt;  // this thread's first group start (nbt: none)
#pragma unroll
    for (uint32_t e = 0; e < P; e++) {
        const uint32_t b = t * P + e, pb = b ? b - 1 : 0u;
        gs[e] = b == 0 || b == half || sz[e] > H || st[b] - st[pb] > H || st[b] / H != st[pb] / H;
        if (gs[e] && lo == nbt) lo = b;
    }
    // first group start at or after each thread's buckets: a minimum scan in
    // reverse thread order
    rev[nt - 1 - t] = lo;
    __syncthreads();
    const uint32_t suf = block_scan(rev[t], MinOp{}, nbt, tmp);  // for thread nt-1-t
    rev[t] = suf;  // block_scan synchronised after every read of rev above
    __syncthreads();
    const uint32_t after = t + 1 < nt ? rev[nt - 2 - t] : nbt;  // first group start past this thread's buckets
    const uint32_t nxt[P] = {gs[1] ? t * P + 1 : after, after};
    uint32_t nc[P], csum = 0;
#pragma unroll
    for (uint32_t e = 0; e < P; e++) {
        const uint32_t b = t * P + e;
        nc[e] = sz[e] > H ? (sz[e] + K - 1) / K : (gs[e] && st[nxt[e]] > st[b] ? 1u : 0u);
        csum += nc[e];
    }
    if (t == 0) nbig = 0;
    uint32_t c0 = block_scan(csum, AddOp{}, 0u, tmp) - csum;  // chunk prefix (its barriers order nbig = 0)
#pragma unroll
    for (uint32_t e = 0; e < P; e++) {
        const uint32_t b = t * P + e, del = b >= half ? 1u : 0u;
        if (sz[e] > H) {
            // a hot bucket's many chunks are written by the whole workgroup below
            uint32_t slot = kBigList;
            if (nc[e] > kBigChunks) slot = atomicAdd(&nbig, 1u);
            if (slot < kBigList) {
                big_b[slot] = b;
                big_c0[slot] = c0;
            } else {
                const uint32_t whole = nc[e] == 1 ? b + 1 : b;  // a bucket split over chunks is held whole by none
                for (uint32_t q = 0; q < nc[e]; q++)
                    chunks[c0 + q] = MergeChunk{st[b] + q * K, min(K, sz[e] - q * K), del, b, whole};
            }
        } else if (nc[e]) {
            chunks[c0] = MergeChunk{st[b], st[nxt[e]] - st[b], del, b, nxt[e]};
        }
        c0 += nc[e];
        meta->chunk0[b + 1] = c0;
    }
    if (t == 0) {
        meta->chunk0[0] = 0;
        meta->n_ins = 0;
        meta->n_del = 0;
    }
    __syncthreads();
    const uint32_t nl = min(nbig, kBigList);
    for (uint32_t l = 0; l < nl; l++) {
        const uint32_t b = big_b[l], cb = big_c0[l], size = st[b + 1] - st[b];
        const uint32_t n = (size + K - 1) / K, del = b >= half ? 1u : 0u;
        for (uint32_t q = t; q < n; q += nt) chunks[cb + q] = MergeChunk{st[b] + q * K, min(K, size - q * K), del, b, b};
    }
}

template <int KB, bool G>
__global__ __launch_bounds__(2 * kMaxBuckets / kStartPer) void k_part_start(MergeMeta* __restrict__ meta,
                                                                            MergeChunk* __restrict__ chunks) {
    part_start_block<KB, G>(meta, chunks);
}

// Scatters the keys into their buckets (order inside a bucket is free).
// uint32 keys are first sorted by bucket inside the group (LDS), so that the
// group writes each bucket's keys as one contiguous run; wider keys go
// straight to their slots.
// One partition tile, block blk of ntiles.  LOCAL_STARTS: the bucket starts
// come from a scan of the bucket totals here, not from k_part_start.
template <int KB, bool G, class P, uint32_t OPS, bool LOCAL_STARTS>
__device__ __forceinline__ void part_scatter_tile(const P& plan, const uint32_t* __restrict__ offs,
                                                  const MergeMeta* __restrict__ meta,
                                                  MKey<KB, G>* __restrict__ part, uint32_t nb_log2, uint32_t blk,
                                                  uint32_t ntiles) {
    constexpr uint32_t R = OPS / kPartThreads;  // keys per thread
    constexpr bool kStage = sizeof(MKey<KB, G>) <= 8;
    __shared__ uint32_t hist[2 * kMaxBuckets];       // local counts, then the group's first global slot
    __shared__ uint32_t lstart[2 * kMaxBuckets];     // exclusive prefix of the local counts
    __shared__ uint32_t tmp[16];
    __shared__ MKey<KB, G> stage[kStage ? OPS : 1];
    __shared__ uint16_t sbk[kStage ? OPS : 1];
    const uint32_t nbt = 2u << nb_log2;
    const Work w = plan.at(blk, OPS);
    MKey<KB, G> k[R];
    bool del[R];
    uint32_t bk[R], rank[R];
    for (uint32_t b = threadIdx.x; b < nbt; b += kPartThreads) hist[b] = 0;
    if (w.count) load_tile_keys<KB, G, R>(w, k, del);
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < R; r++) {
        const uint32_t t = r * kPartThreads + threadIdx.x;
        bk[r] = 0;
        rank[r] = 0;
        if (t < w.count) {
            bk[r] = bucket_of<KB, G>(k[r], del[r], nb_log2, w.g);
            rank[r] = atomicAdd(&hist[bk[r]], 1u);   // place among the group's keys of the bucket
        }
    }
    __syncthreads();
    if constexpr (kStage) {
        // exclusive prefix of the local counts: thread t owns buckets kPer*t ..
        constexpr uint32_t kPer = 2 * kMaxBuckets / kPartThreads;
        const uint32_t t = threadIdx.x;
        uint32_t v[kPer], sum = 0;
#pragma unroll
        for (uint32_t e = 0; e < kPer; e++) {
            const uint32_t b = t * kPer + e;
            v[e] = b < nbt ? hist[b] : 0u;
            sum += v[e];
        }
        uint32_t run = block_scan(sum, AddOp{}, 0u, tmp) - sum;
#pragma unroll
        for (uint32_t e = 0; e < kPer; e++) {
            lstart[t * kPer + e] = run;
            run += v[e];
        }
        const uint32_t row = xcd_row(blk, ntiles);
        if constexpr (LOCAL_STARTS) {
            // nbt = 2 * kPartThreads: thread t owns buckets 2t and 2t + 1
            const uint32_t a0 = meta->total[2 * t], a1 = meta->total[2 * t + 1];
            __syncthreads();  // tmp is free again (the scan above read it)
            const uint32_t ex = block_scan(a0 + a1, AddOp{}, 0u, tmp) - (a0 + a1);
            hist[2 * t] = ex + offs[size_t(row) * nbt + 2 * t];
            hist[2 * t + 1] = ex + a0 + offs[size_t(row) * nbt + 2 * t + 1];
        } else {
            for (uint32_t b = t; b < nbt; b += kPartThreads) hist[b] = meta->start[b] + offs[size_t(row) * nbt + b];
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < R; r++) {
            const uint32_t t = r * kPartThreads + threadIdx.x;
            if (t < w.count) {
                const uint32_t i = lstart[bk[r]] + rank[r];
                stage[i] = k[r];
                sbk[i] = uint16_t(bk[r]);
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < w.count; i += kPartThreads) {
            const uint32_t bb = sbk[i];
            part[hist[bb] + (i - lstart[bb])] = stage[i];
        }
    } else {
        __syncthreads();
        const uint32_t row = xcd_row(blk, ntiles), t = threadIdx.x;
        if constexpr (LOCAL_STARTS) {
            const uint32_t a0 = meta->total[2 * t], a1 = meta->total[2 * t + 1];
            const uint32_t ex = block_scan(a0 + a1, AddOp{}, 0u, tmp) - (a0 + a1);
            hist[2 * t] = ex + offs[size_t(row) * nbt + 2 * t];
            hist[2 * t + 1] = ex + a0 + offs[size_t(row) * nbt + 2 * t + 1];
        } else {
            for (uint32_t b = t; b < nbt; b += kPartThreads) hist[b] = meta->start[b] + offs[size_t(row) * nbt + b];
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < R; r++) {
            const uint32_t t = r * kPartThreads + threadIdx.x;
            if (t < w.count) part[hist[bk[r]] + rank[r]] = k[r];
        }
    }
}

template <int KB, bool G, class P, uint32_t OPS = kPartOps>
__global__ __launch_bounds__(kPartThreads) void k_part_scatter(P plan, const uint32_t* __restrict__ offs,
                                                               const MergeMeta* __restrict__ meta,
                                                               MKey<KB, G>* __restrict__ part, uint32_t nb_log2) {
    part_scatter_tile<KB, G, P, OPS, false>(plan, offs, meta, part, nb_log2, blockIdx.x, gridDim.x);
}

// A lone sketch's batch with all 2 * kMaxBuckets buckets of staged uint32
// keys: the last workgroup lays the buckets and merge chunks out (as
// k_part_start does), the others scatter their tiles with the bucket starts
// scanned from the totals themselves, so no launch sits between the column
// scan and the scatter.  Neither side reads what the other writes.
template <int KB, class P, uint32_t OPS>
__global__ __launch_bounds__(kPartThreads) void k_part_scatter_start(P plan, const uint32_t* __restrict__ offs,
                                                                     MergeMeta* __restrict__ meta,
                                                                     MergeChunk* __restrict__ chunks,
                                                                     MKey<KB, false>* __restrict__ part,
                                                                     uint32_t nb_log2, uint32_t ntiles) {
    static_assert(2 * kMaxBuckets / kStartPer == kPartThreads, "the layout workgroup is a partition workgroup");
    if (blockIdx.x == ntiles) {
        part_start_block<KB, false>(meta, chunks);
        return;
    }
    part_scatter_tile<KB, false, P, OPS, true>(plan, offs, meta, part, nb_log2, blockIdx.x, ntiles);
}

// Merges one chunk and emits its entries (key, count).  cap = entry capacity
// (insert entries at [0, n_ins), delete entries at [cap - n_del, cap)).
//
// A lone sketch's bucket is a range of row-0 cells, so an insert chunk that
// holds its buckets whole is the only workgroup of the batch touching their
// row-0 records.  If their Fat counters fit the LDS table and its entries
// are at least one per 8 of those counters, the chunk takes row 0's S1
// (snapshot) and S2 (Fat +) in place: it reads the snapshot of
// its entries, then, after a barrier, sums their counts per counter in LDS
// and adds the sums with plain stores.  Its entries carry kRow0Done, and the
// entry kernels skip row 0 for them.
template <int KB, bool G, class SR>
__global__ __launch_bounds__((MergeShape<KB, G>::kThreads)) void k_merge(const MKey<KB, G>* __restrict__ part,
                                                  MergeMeta* __restrict__ meta,
                                                  const MergeChunk* __restrict__ chunks,
                                                  MKey<KB, G>* __restrict__ ent_key,
                                                  uint32_t* __restrict__ ent_cnt, uint32_t cap, uint32_t nb_log2,
                                                  SR sr, uint32_t* __restrict__ bpre,
                                                  uint16_t* __restrict__ asnap, uint32_t row0) {
    constexpr int J = MergeShape<KB, G>::J;
    constexpr uint32_t kThreads = MergeShape<KB, G>::kThreads;
    constexpr uint32_t kSlots = MergeShape<KB, G>::kSlots;
    __shared__ MergeLDS<KB, G> L;
    __shared__ uint32_t nloc, base;
    const uint32_t nbt = 2u << nb_log2;
    const uint32_t c = blockIdx.x;
    if (c >= meta->chunk0[nbt]) return;
    const MergeChunk ck = chunks[c];
    const bool del = ck.del != 0;
    const uint32_t first = ck.first, n = ck.n;
    bool inplace = false;                         // row 0's S1 and S2 taken here (same for the workgroup)
    uint32_t lo = 0, ncnt = 0;                    // first row-0 cell of the chunk's buckets, their Fat counters
    SketchDesc sd{};
    if constexpr (!G) {
        sd = sr.of(0u);
        const uint64_t w = sd.g.w, round = (1ull << nb_log2) - 1;
        lo = uint32_t((uint64_t(ck.b_lo) * w + round) >> nb_log2);  // bucket b: cells with h * nb / w = b
        const uint32_t hi = uint32_t((uint64_t(ck.b_hi) * w + round) >> nb_log2);
        ncnt = (hi - lo) * sd.g.z;
        inplace = row0 && !del && ck.b_hi > ck.b_lo && uint64_t(hi - lo) * sd.g.z <= kSlots;
    }
    // about two slots per key (at least one per thread): a small chunk clears
    // and probes a small table
    const uint32_t slots = min(kSlots, max(kThreads, 2 * n));
    // the chunk's keys in flight before any is used (slots past its end load
    // its first key and stay invalid)
    MKey<KB, G> k[J] = {};
    if (n) {
#pragma unroll
        for (int j = 0; j < J; j++) {
            const uint32_t idx = uint32_t(j) * kThreads + threadIdx.x;
            k[j] = part[first + (idx < n ? idx : 0u)];
        }
    }
    for (uint32_t i = threadIdx.x; i < slots; i += kThreads) L.slot[i] = kEmpty;
    if (threadIdx.x == 0) nloc = 0;
#pragma unroll
    for (int j = 0; j < J; j++) {
        const uint32_t idx = uint32_t(j) * kThreads + threadIdx.x;
        if (idx < n) L.key[idx] = k[j];
    }
    __syncthreads();
    uint32_t made[J];                             // slots this thread created (one per new key)
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < J; j++) {
        const uint32_t idx = uint32_t(j) * kThreads + threadIdx.x;
        const uint32_t wgt = wave_peel<kPeel>(k[j], idx < n, [](const MKey<KB, G>& a, const MKey<KB, G>& b) {
            return mkey_eq<KB, G>(a, b);
        });
        made[j] = wgt ? merge_insert<KB, G>(L, k[j], idx, wgt, slots) : kEmpty;
        mine += made[j] != kEmpty;
    }
    // The creator of a slot emits its entry: a wavefront prefix sum of the
    // creators' counts, one LDS atomic per wavefront, one global atomic per group.
    uint32_t incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t x = __shfl_up(incl, off);
        if (int(lane_id()) >= off) incl += x;
    }
    uint32_t wbase = 0;
    if (lane_id() == 63u) wbase = atomicAdd(&nloc, incl);
    wbase = __shfl(wbase, 63);
    __syncthreads();                              // every count final, nloc complete
    if (threadIdx.x == 0) base = atomicAdd(del ? &meta->n_del : &meta->n_ins, nloc);
    // in place only where the entries are dense enough to repay clearing and
    // scanning the per-counter table (at least one per 8 counters)
    inplace = inplace && uint64_t(nloc) * 8 >= ncnt;
    __syncthreads();
    uint32_t rank = base + wbase + incl - mine;
    uint32_t eid[J], ecnt[J];
#pragma unroll
    for (int j = 0; j < J; j++) {
        if (made[j] == kEmpty) continue;
        const uint32_t id = del ? cap - 1 - rank : rank;
        rank++;
        eid[j] = id;
        ecnt[j] = L.slot[made[j]] & 0xffffu;
        ent_key[id] = k[j];
        ent_cnt[id] = ecnt[j] | (inplace ? kRow0Done : 0u);
    }
    if constexpr (!G) {
        if (inplace) {
            const uint32_t z = sd.g.z;
            __syncthreads();                      // every count has been read from the table
            for (uint32_t i = threadIdx.x; i < ncnt; i += kThreads) L.slot[i] = 0;
            __syncthreads();
            // every snapshot gather in flight before any is stored (a thread
            // without the entry reads cell 0 and drops it)
            uint32_t hc[J], fc[J], sa[J], sb[J];
#pragma unroll
            for (int j = 0; j < J; j++) {
                split(sd.g, Mixed<KB>(k[j].k).row(sd.g.seed_base), hc[j], fc[j]);
                const bool e = made[j] != kEmpty;
                const uint32_t* rec = sd.fat + size_t(e ? hc[j] : 0u) * sd.g.rs;  // row 0
                sa[j] = rec[z];
                sb[j] = rec[e ? fc[j] : 0u];
            }
#pragma unroll
            for (int j = 0; j < J; j++) {
                if (made[j] == kEmpty) continue;
                asnap[eid[j]] = uint16_t(sa[j]);
                bpre[eid[j]] = sb[j];
                atomicAdd(&L.slot[(hc[j] - lo) * z + fc[j]], ecnt[j]);
            }
            __syncthreads();                      // every snapshot read before a counter moves
            for (uint32_t i = threadIdx.x; i < ncnt; i += kThreads) {
                const uint32_t v = L.slot[i];
                if (v) sd.fat[size_t(lo + i / z) * sd.g.rs + i % z] += v;
            }
        }
    }
}

// Where an entry's sketch lives: one sketch, or a table of them.  take(s):
// whether the entry kernels serve sketch s's entries (all of them, except
// in a sketch table's sub-round that also has owner-computed sketches:
// SketchSide then leaves to the owner path every sketch with ranges).
struct OneSketch {
    Geom g;
    uint32_t* fat;
    uint32_t* slim;
    __device__ __forceinline__ SketchDesc of(uint32_t) const { return SketchDesc{g, fat, slim}; }
    __device__ __forceinline__ bool take(uint32_t) const { return true; }
};
struct SketchTable {
    const SketchDesc* t;
    __device__ __forceinline__ SketchDesc of(uint32_t s) const { return t[s]; }
    __device__ __forceinline__ bool take(uint32_t) const { return true; }
};
struct SketchSide {
    const SketchDesc* t;
    const uint32_t* qbase;  // the sub-round's first range of each sketch, ~0: none (atomic path)
    __device__ __forceinline__ SketchDesc of(uint32_t s) const { return t[s]; }
    __device__ __forceinline__ bool take(uint32_t s) const { return qbase[s] == ~0u; }
};

// S1 over merged insert entries: Slim and Fat counters before the batch.
template <int KB, int D, bool G, class SR>
__global__ __launch_bounds__(kBlock) void k_entries_snapshot(const MergeMeta* __restrict__ meta,
                                                             const MKey<KB, G>* __restrict__ ent_key,
                                                             const uint32_t* __restrict__ ent_cnt, SR sr,
                                                             uint32_t* __restrict__ bpre,
                                                             uint16_t* __restrict__ asnap, uint32_t stride) {
    constexpr int R = D ? D : kMaxD;
    const uint32_t n = meta->n_ins;
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < n; e += gridDim.x * kBlock) {
        const MKey<KB, G> m = ent_key[e];
        if (!sr.take(mkey_sketch<KB, G>(m))) continue;
        const SketchDesc sd = sr.of(mkey_sketch<KB, G>(m));
        const uint32_t d = SF_ROWS(D, sd.g);
        const uint32_t i0 = ent_cnt[e] & kRow0Done ? 1u : 0u;  // row 0 taken by the merge
        const Mixed<KB> mx(m.k);
        uint32_t av[R], bv[R];
#pragma unroll
        for (int i = 0; i < R; i++) {
            if (uint32_t(i) < d && uint32_t(i) >= i0) {
                uint32_t h, f;
                split(sd.g, mx.row(sd.g.seed_base + i), h, f);
                const size_t cell = size_t(i) * sd.g.w + h;
                av[i] = sd.slim[cell * sd.g.rs];     // same record as the Fat counter below
                bv[i] = sd.fat[cell * sd.g.rs + f];
            }
        }
#pragma unroll
        for (int i = 0; i < R; i++) {
            if (uint32_t(i) < d && uint32_t(i) >= i0) {
                asnap[size_t(i) * stride + e] = uint16_t(av[i]);
                bpre[size_t(i) * stride + e] = bv[i];
            }
        }
    }
}

// S2 / S4 over merged entries: one atomic per entry and row carrying its count.
template <int KB, int D, bool G, class SR>
__global__ __launch_bounds__(kBlock) void k_entries_fat(MergeMeta* __restrict__ meta,
                                                        const MKey<KB, G>* __restrict__ ent_key,
                                                        const uint32_t* __restrict__ ent_cnt, uint32_t cap,
                                                        SR sr, uint32_t del) {
    const uint32_t n = del ? meta->n_del : meta->n_ins;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(del ? &meta->acc_del : &meta->acc_ins, (unsigned long long)n);
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < n; e += gridDim.x * kBlock) {
        const uint32_t id = del ? cap - 1 - e : e;
        const uint32_t raw = ent_cnt[id], cnt = raw & ~kRow0Done;
        const uint32_t v = del ? 0u - cnt : cnt;
        const uint32_t i0 = raw & kRow0Done ? 1u : 0u;  // row 0 added by the merge
        const MKey<KB, G> m = ent_key[id];
        if (!sr.take(mkey_sketch<KB, G>(m))) continue;
        const SketchDesc sd = sr.of(mkey_sketch<KB, G>(m));
        const uint32_t d = SF_ROWS(D, sd.g);
        const Mixed<KB> mx(m.k);
#pragma unroll
        for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
            if (i < d && i >= i0) {
                uint32_t h, f;
                split(sd.g, mx.row(sd.g.seed_base + i), h, f);
                atomic_add_u32(&sd.fat[(size_t(i) * sd.g.w + h) * sd.g.rs + f], v);
            }
        }
    }
}

// S3 over merged insert entries.
template <int KB, int D, bool G, class SR>
__global__ __launch_bounds__(kBlock) void k_entries_raise(const MergeMeta* __restrict__ meta,
                                                          const MKey<KB, G>* __restrict__ ent_key, SR sr,
                                                          const uint32_t* __restrict__ bpre,
                                                          const uint16_t* __restrict__ asnap, uint32_t stride) {
    constexpr int R = D ? D : kMaxD;
    const uint32_t n = meta->n_ins;
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < n; e += gridDim.x * kBlock) {
        const MKey<KB, G> m = ent_key[e];
        if (!sr.take(mkey_sketch<KB, G>(m))) continue;
        const SketchDesc sd = sr.of(mkey_sketch<KB, G>(m));
        const uint32_t d = SF_ROWS(D, sd.g);
        const Mixed<KB> mx(m.k);
        size_t cell[R];
        uint32_t cur[R];
        uint32_t m0 = ~0u, bmin = ~0u, delta = ~0u;
#pragma unroll
        for (int i = 0; i < R; i++) {
            cell[i] = 0;
            cur[i] = kSlimMax;
            if (uint32_t(i) < d) {
                uint32_t h, f;
                split(sd.g, mx.row(sd.g.seed_base + i), h, f);
                cell[i] = size_t(i) * sd.g.w + h;
                const uint32_t* rec = sd.fat + cell[i] * sd.g.rs;
                const uint32_t post = rec[f];
                cur[i] = rec[sd.g.z];  // the Slim word of the same record: no extra line
                const uint32_t grew = post - bpre[size_t(i) * stride + e];
                m0 = min(m0, uint32_t(asnap[size_t(i) * stride + e]));
                bmin = min(bmin, post);
                delta = min(delta, grew);
            }
        }
        const uint64_t rise = uint64_t(m0) + delta;
        const uint64_t level = m0 > bmin ? m0 : bmin;
        const uint64_t tt = rise < level ? rise : level;
        const uint32_t T = uint32_t(tt < kSlimMax ? tt : kSlimMax);
        // Slim words only grow during S3 and cur is at least the snapshot, so a
        // cell already at T or above (raised by another entry) needs no atomic.
#pragma unroll
        for (int i = 0; i < R; i++)
            if (uint32_t(i) < d && cur[i] < T) atomic_max_u32(&sd.slim[cell[i] * sd.g.rs], T);
    }
}

// S5 over merged delete entries.
template <int KB, int D, bool G, class SR>
__global__ __launch_bounds__(kBlock) void k_entries_clamp(const MergeMeta* __restrict__ meta,
                                                          const MKey<KB, G>* __restrict__ ent_key, uint32_t cap,
                                                          SR sr) {
    const uint32_t n = meta->n_del;
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < n; e += gridDim.x * kBlock) {
        const MKey<KB, G> m = ent_key[cap - 1 - e];
        if (!sr.take(mkey_sketch<KB, G>(m))) continue;
        const SketchDesc sd = sr.of(mkey_sketch<KB, G>(m));
        const uint32_t d = SF_ROWS(D, sd.g);
        const Mixed<KB> mx(m.k);
#pragma unroll
        for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
            if (i < d) {
                uint32_t h, f;
                split(sd.g, mx.row(sd.g.seed_base + i), h, f);
                const size_t cell = size_t(i) * sd.g.w + h;
                const uint32_t mval = bucket_max(sd.fat, cell, sd.g);
                if (sd.slim[cell * sd.g.rs] > mval) atomic_min_u32(&sd.slim[cell * sd.g.rs], mval);
            }
        }
    }
}

// S1 one row per XCD.  Its rows are independent (it stores per-row values),
// so with D dividing 8 workgroup b handles row (b mod 8) mod D for its share
// of the entries, and an XCD's random reads stay within one row of records (a
// quarter of the footprint at D = 4, so more of them hit its L2).  As with the
// query, the dispatch order only decides cache hits.  gridDim.x is a multiple
// of 8.  (S5 gains nothing from this: a batch has few delete entries, and the
// wider grid costs more than the cache hits save.)
struct XcdRow {
    uint32_t r, slot, nslots;
    template <int D> __device__ __forceinline__ static XcdRow of() {
        static_assert(D > 0 && kXcds % D == 0, "D must divide the XCD count");
        const uint32_t x = blockIdx.x % kXcds, nsub = kXcds / D;
        return XcdRow{x % D, (blockIdx.x / kXcds) * nsub + x / D, (gridDim.x / kXcds) * nsub};
    }
};

template <int KB, int D, bool G, class SR>
__global__ __launch_bounds__(kBlock) void k_entries_snapshot_rows(const MergeMeta* __restrict__ meta,
                                                                  const MKey<KB, G>* __restrict__ ent_key,
                                                                  const uint32_t* __restrict__ ent_cnt, SR sr,
                                                                  uint32_t* __restrict__ bpre,
                                                                  uint16_t* __restrict__ asnap, uint32_t stride) {
    const XcdRow xr = XcdRow::of<D>();
    const uint32_t n = meta->n_ins;
    for (uint32_t e = xr.slot * kBlock + threadIdx.x; e < n; e += xr.nslots * kBlock) {
        if (xr.r == 0 && (ent_cnt[e] & kRow0Done)) continue;  // row 0 taken by the merge
        const MKey<KB, G> m = ent_key[e];
        if (!sr.take(mkey_sketch<KB, G>(m))) continue;
        const SketchDesc sd = sr.of(mkey_sketch<KB, G>(m));
        uint32_t h, f;
        split(sd.g, Mixed<KB>(m.k).row(sd.g.seed_base + xr.r), h, f);
        const size_t cell = size_t(xr.r) * sd.g.w + h;
        const uint32_t a = sd.slim[cell * sd.g.rs];  // same record as the Fat counter
        const uint32_t b = sd.fat[cell * sd.g.rs + f];
        asnap[size_t(xr.r) * stride + e] = uint16_t(a);
        bpre[size_t(xr.r) * stride + e] = b;
    }
}

}  // namespace sfk
