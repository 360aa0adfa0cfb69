// Owner-computes S1..S5 on the batch-wide merge path (a lone sketch, or the
// sub-rounds of a sketch table).
//
// After the merge each entry (a distinct key of a merge chunk, with its
// count) touches one cell in each of the d rows.  Instead of d random record
// reads and d device-scope atomics per entry and step, the (entry, row) pairs
// are partitioned by (op type, row, cell range).  Each range of 2^cr_shift
// consecutive cells of a row has one owning workgroup per step, which is then
// the only one reading or writing those records: it stages the range's Fat
// buckets and Slim words in LDS, applies the step there with LDS atomics and
// writes the range back with coalesced stores.
//
//   k_pair_count    per tile of entries and row: pairs per column in LDS
//   k_pair_colscan  each tile's offset inside every column; column totals
//   k_pair_start    column starts
//   k_pair_scatter  per tile and row: counting sort in LDS, pairs written in
//                   runs; for insert entries the position of the pair of
//                   each row goes to pos[row][entry]
//   k_own_step      per (row, range), its records staged in LDS: S3 + S4 +
//                   S5 of the previous batch, then S1 + S2 of this one; every
//                   insert pair gets, in pair order, its Slim counter before
//                   the batch, its Fat counter's growth over the batch and
//                   the counter after it
//   k_level         per insert entry: T = min(m0 + delta, max(m0, Bmin),
//                   65535) from its d pairs, gathered through pos (the pairs
//                   of one tile sit in short runs, so one fetched line serves
//                   several of the tile's entries)
// The last batch of an update call ends with a k_own_step that has no next
// batch.  A lone sketch runs the partition, merge and pair kernels of batch
// k + 1 on a second stream while k_own_step and k_level of batch k run: they
// read keys and entries only, and the buffers the two sides share are kept
// apart (three sets of column starts, two of pairs; k_pair_scatter of batch
// k + 1, which writes pairs and pos, waits for k_level of batch k).
//
// Same results as the entry kernels of sf_kernels.hpp, bit for bit: S2 and S4
// are sums, S3 a maximum and S5 a minimum per cell, and every pair of a key
// sees the same snapshot.
#pragma once

#include "sf_kernels.hpp"

namespace sfk {

// Entries per partitioning tile: about kPairTiles tiles per batch, between
// kPairTileMin and kPairTileMax entries each, so that few entries still spread
// over many workgroups and many entries still write runs of several pairs.
constexpr uint32_t kPairTileMin = 512, kPairTileMax = 4096, kPairTiles = 256;
constexpr uint32_t kPairThreads = 512;   // threads of the per-tile kernels
constexpr uint32_t kCountThreads = 256;  // threads of k_pair_count
constexpr uint32_t kMaxCols = 16384;     // columns: 2 op types x d rows x R ranges
constexpr uint32_t kMaxRanges = 1024;    // ranges per row
constexpr uint32_t kOwnCounters = 8192;  // Fat counters of one range (its records fit 64 KiB of LDS)
constexpr uint32_t kOwnThreads = 256;    // threads of an owner workgroup ...
constexpr uint32_t kOwnThreadsWide = 512;  // ... whose range takes more than kOwnWideLds bytes of LDS
constexpr size_t kOwnWideLds = 24u << 10;

__host__ __device__ constexpr uint32_t pair_tile(uint32_t nv) {
    const uint32_t per = (nv + kPairTiles - 1) / kPairTiles;
    const uint32_t t = (per + kPairTileMin - 1) / kPairTileMin * kPairTileMin;
    return t < kPairTileMin ? kPairTileMin : t > kPairTileMax ? kPairTileMax : t;
}
// Tiles (grid width) that cover every entry count up to cap.
// A multiple of 8, so that in the (tile, row) grids tile b runs on XCD b % 8
// whatever its row.
__host__ __device__ constexpr uint32_t pair_tiles_max(uint32_t cap) {
    const uint32_t big = ((cap + kPairTileMax - 1) / kPairTileMax + 7) / 8 * 8;
    return big > kPairTiles ? big : kPairTiles;
}

struct OwnerGeom {
    uint32_t R;         // cell ranges per row (a sketch table: of every sketch of the sub-round)
    uint32_t cr_shift;  // log2(cells per range)
    uint32_t zbits;     // bits of the slot in a pair's local code (2^zbits >= z)
    uint32_t ncol;      // 2 * d * R: insert columns (row-major), then delete columns
    uint32_t xcd;       // owner workgroup b takes row (b % 8) % d
    uint32_t d;         // rows (the same for every sketch of a table)
};

// Which range (per row) a cell of a sketch belongs to, and back.  A lone
// sketch's ranges are its own: range = cell >> cr_shift.  In a sketch table
// the ranges of one sub-round's sketches are numbered one after the other
// (the same numbering in every row): qbase[s] is sketch s's first, and range
// q belongs to sketch qsk[q], where it is the qr[q]-th.
struct LoneRanges {
    __device__ __forceinline__ bool has(uint32_t) const { return true; }
    __device__ __forceinline__ uint32_t q_of(uint32_t, uint32_t rng) const { return rng; }
    __device__ __forceinline__ void range_of(uint32_t q, uint32_t& sketch, uint32_t& r) const {
        sketch = 0;
        r = q;
    }
};
struct TableRanges {
    const uint32_t* qbase;
    const uint32_t* qsk;
    const uint32_t* qr;
    // whether sketch s is owner-computed in this sub-round (else its entries
    // take the atomic entry kernels)
    __device__ __forceinline__ bool has(uint32_t s) const { return qbase[s] != ~0u; }
    __device__ __forceinline__ uint32_t q_of(uint32_t s, uint32_t rng) const { return qbase[s] + rng; }
    __device__ __forceinline__ void range_of(uint32_t q, uint32_t& sketch, uint32_t& r) const {
        sketch = qsk[q];
        r = qr[q];
    }
};

struct PairMeta {
    uint32_t total[kMaxCols];      // pairs per column
    uint32_t start[kMaxCols + 1];  // first pair of each column; [ncol] = all pairs
    uint32_t n_ins, n_del;         // the batch's insert and delete entries (copied from the merge)
};

// A pair: entry index (low word); local code (cell in range << zbits | slot)
// and the entry's count in the high word.  Counts fit 16 bits: an entry
// merges the copies of a key inside one merge chunk, which holds at most
// MergeShape::kChunk keys.
static_assert(MergeShape<4, false>::kChunk < 65536 && MergeShape<13, false>::kChunk < 65536,
              "an entry's count must fit a pair's 16-bit count field");
__device__ __forceinline__ uint64_t make_pair(uint32_t e, uint32_t code, uint32_t count) {
    return uint64_t(e) | (uint64_t(code | (count << 16)) << 32);
}

// The (row, range) an owner workgroup takes.  With xcd, workgroup b runs on
// XCD b % 8 (round-robin dispatch), so each XCD's L2 sees one row's records
// only; placement decides cache hits, never results.
__device__ __forceinline__ void owner_of(const OwnerGeom& og, uint32_t d, uint32_t& row, uint32_t& range) {
    const uint32_t b = blockIdx.x;
    if (og.xcd) {
        const uint32_t x = b % kXcds;
        row = x % d;
        range = (b / kXcds) * (kXcds / d) + x / d;
    } else {
        row = b / og.R;
        range = b % og.R;
    }
}

// Entry of virtual index v: inserts are entries [0, ni), deletes sit at
// cap-1, cap-2, ... (the merge fills them from the end).
__device__ __forceinline__ uint32_t entry_of(uint32_t v, uint32_t ni, uint32_t cap) {
    return v < ni ? v : cap - 1 - (v - ni);
}

// Pairs of one row of one tile per column (blockIdx.y = row).
template <int KB, bool G, class SR, class RM>
__global__ __launch_bounds__(kCountThreads) void k_pair_count(const MergeMeta* __restrict__ meta,
                                                              const MKey<KB, G>* __restrict__ ent_key,
                                                              uint32_t cap, SR sr, RM rm, OwnerGeom og,
                                                              uint32_t* __restrict__ hmat) {
    __shared__ uint32_t hist[2 * kMaxRanges];
    const uint32_t ni = meta->n_ins, nv = ni + meta->n_del, T = pair_tile(nv);
    const uint32_t lo = blockIdx.x * T;
    if (lo >= nv) return;
    const uint32_t hi = min(nv, lo + T), i = blockIdx.y, R = og.R, d = og.d;
    for (uint32_t c = threadIdx.x; c < 2 * R; c += kCountThreads) hist[c] = 0;
    __syncthreads();
    for (uint32_t v = lo + threadIdx.x; v < hi; v += kCountThreads) {
        const MKey<KB, G> m = ent_key[entry_of(v, ni, cap)];
        const uint32_t sk = mkey_sketch<KB, G>(m);
        if (!rm.has(sk)) continue;
        const Geom g = sr.of(sk).g;
        uint32_t h, f;
        split(g, Mixed<KB>(m.k).row(g.seed_base + i), h, f);
        atomicAdd(&hist[(v < ni ? 0u : R) + rm.q_of(sk, h >> og.cr_shift)], 1u);
    }
    __syncthreads();
    uint32_t* out = hmat + size_t(xcd_row(blockIdx.x, (nv + T - 1) / T)) * og.ncol + i * R;
    for (uint32_t c = threadIdx.x; c < 2 * R; c += kCountThreads) out[c < R ? c : d * R + c - R] = hist[c];
}

// Column scans of the histogram matrix over the tiles that hold entries: 64
// columns per workgroup, a wavefront reading 256 contiguous bytes of a row.
// (Taking the column starts in the workgroup that finishes last costs more
// than a launch: making the totals visible across XCDs writes back the L2.)
template <int = 0>
__global__ __launch_bounds__(kScanCols * kScanWaves) void k_pair_colscan(uint32_t* __restrict__ hmat,
                                                                         const MergeMeta* __restrict__ meta,
                                                                         PairMeta* __restrict__ pm, uint32_t ncol) {
    const uint32_t nv = meta->n_ins + meta->n_del, T = pair_tile(nv);
    colscan_wide<uint32_t>(hmat, (nv + T - 1) / T, ncol, pm->total);
}

// Column starts: one workgroup, thread t owns columns kPer*t ...  Also keeps
// the batch's entry counts beside them (the merge metadata is the next
// batch's once its partition starts) and adds them to the merge statistics.
template <int = 0>
__global__ __launch_bounds__(1024) void k_pair_start(PairMeta* __restrict__ pm, uint32_t ncol,
                                                     MergeMeta* __restrict__ meta, uint32_t add_stats) {
    constexpr uint32_t kPer = kMaxCols / 1024;
    __shared__ uint32_t tmp[16];
    uint32_t v[kPer], sum = 0;
#pragma unroll
    for (uint32_t e = 0; e < kPer; e++) {
        const uint32_t c = threadIdx.x * kPer + e;
        v[e] = c < ncol ? pm->total[c] : 0u;
        sum += v[e];
    }
    uint32_t run = block_scan(sum, AddOp{}, 0u, tmp) - sum;
#pragma unroll
    for (uint32_t e = 0; e < kPer; e++) {
        const uint32_t c = threadIdx.x * kPer + e;
        if (c < ncol) pm->start[c] = run;
        run += v[e];
    }
    if (threadIdx.x == 1023) pm->start[ncol] = run;
    if (threadIdx.x == 0) {
        pm->n_ins = meta->n_ins;
        pm->n_del = meta->n_del;
        if (add_stats) {  // (else the entry kernels of the same sub-round count them)
            meta->acc_ins += meta->n_ins;
            meta->acc_del += meta->n_del;
        }
    }
}

// Writes the pairs of one row (blockIdx.y) of one tile into their columns:
// counted per (op type, range) in LDS, staged in column order, written out as
// one run per column.  For insert entries, the position of the pair goes to
// pos[row][entry].
template <int KB, bool G, class SR, class RM>
__global__ __launch_bounds__(kPairThreads) void k_pair_scatter(const MergeMeta* __restrict__ meta,
                                                               const MKey<KB, G>* __restrict__ ent_key,
                                                               const uint32_t* __restrict__ ent_cnt,
                                                               uint32_t cap, SR sr, RM rm, OwnerGeom og,
                                                               const uint32_t* __restrict__ hmat,
                                                               const PairMeta* __restrict__ pm,
                                                               uint64_t* __restrict__ pairs,
                                                               uint32_t* __restrict__ pos, uint32_t pos_stride) {
    constexpr uint32_t E = kPairTileMax / kPairThreads;
    constexpr uint32_t kPer = 2 * kMaxRanges / kPairThreads;  // columns per thread in the scan
    __shared__ uint64_t stage[kPairTileMax];
    __shared__ uint16_t scol[kPairTileMax];   // column (op type * R + range) of each staged pair
    __shared__ uint32_t cnt[2 * kMaxRanges];  // the tile's pairs per column
    __shared__ uint32_t lst[2 * kMaxRanges];  // their first staging slot
    __shared__ uint32_t gb[2 * kMaxRanges];   // their first position in pairs
    __shared__ uint32_t tmp[16];
    const uint32_t ni = meta->n_ins, nv = ni + meta->n_del, T = pair_tile(nv);
    const uint32_t lo = blockIdx.x * T;
    if (lo >= nv) return;
    const uint32_t n = min(nv - lo, T), i = blockIdx.y;
    const uint32_t trow = xcd_row(blockIdx.x, (nv + T - 1) / T);  // this tile's row of hmat
    const uint32_t d = og.d, R = og.R, nc = 2 * R;
    const uint32_t cmask = (1u << og.cr_shift) - 1;
    for (uint32_t c = threadIdx.x; c < nc; c += kPairThreads) cnt[c] = 0;
    uint32_t eid[E], c16[E], col[E], code[E], rank[E];
    bool own[E];  // the entry's sketch is owner-computed (always, for a lone sketch)
    MKey<KB, G> mk[E];
    uint32_t ec[E];
    // every entry's key and count in flight before any is used (slots past
    // the tile's end load its first entry and are skipped below)
#pragma unroll
    for (uint32_t j = 0; j < E; j++) {
        const uint32_t t = j * kPairThreads + threadIdx.x;
        eid[j] = entry_of(lo + (t < n ? t : 0u), ni, cap);
        mk[j] = ent_key[eid[j]];
        ec[j] = ent_cnt[eid[j]];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < E; j++) {
        const uint32_t t = j * kPairThreads + threadIdx.x;
        own[j] = false;
        c16[j] = col[j] = code[j] = rank[j] = 0;
        if (t < n) {
            const MKey<KB, G>& m = mk[j];
            const uint32_t sk = mkey_sketch<KB, G>(m);
            own[j] = rm.has(sk);
            if (own[j]) {
                c16[j] = ec[j] & ~kRow0Done;
                const Geom g = sr.of(sk).g;
                uint32_t h, f;
                split(g, Mixed<KB>(m.k).row(g.seed_base + i), h, f);
                col[j] = (lo + t >= ni ? R : 0u) + rm.q_of(sk, h >> og.cr_shift);
                code[j] = ((h & cmask) << og.zbits) | f;
                rank[j] = atomicAdd(&cnt[col[j]], 1u);
            }
        }
    }
    __syncthreads();
    {  // exclusive scan of the counts; thread t owns columns kPer*t ...
        uint32_t v[kPer], sum = 0;
#pragma unroll
        for (uint32_t e = 0; e < kPer; e++) {
            const uint32_t c = threadIdx.x * kPer + e;
            v[e] = c < nc ? cnt[c] : 0u;
            sum += v[e];
        }
        uint32_t run = block_scan(sum, AddOp{}, 0u, tmp) - sum;
#pragma unroll
        for (uint32_t e = 0; e < kPer; e++) {
            const uint32_t c = threadIdx.x * kPer + e;
            if (c < nc) lst[c] = run;
            run += v[e];
        }
    }
    for (uint32_t c = threadIdx.x; c < nc; c += kPairThreads) {
        const uint32_t gcol = (c < R ? 0u : d * R) + i * R + (c < R ? c : c - R);
        gb[c] = pm->start[gcol] + hmat[size_t(trow) * og.ncol + gcol];
    }
    __syncthreads();
    const uint32_t nst = lst[nc - 1] + cnt[nc - 1];  // pairs staged: the tile's owner-computed entries
#pragma unroll
    for (uint32_t j = 0; j < E; j++) {
        const uint32_t t = j * kPairThreads + threadIdx.x;
        if (t >= n || !own[j]) continue;
        const uint32_t s = lst[col[j]] + rank[j];
        stage[s] = make_pair(eid[j], code[j], c16[j]);
        scol[s] = uint16_t(col[j]);
        if (lo + t < ni) pos[size_t(i) * pos_stride + eid[j]] = gb[col[j]] + rank[j];
    }
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < nst; s += kPairThreads) {
        const uint32_t c = scol[s];
        pairs[gb[c] + (s - lst[c])] = stage[s];
    }
}

// T of every insert entry of tile blk from its d pairs, NT threads.  The
// tiles are those of the pair partition, so the runs its pairs were written
// in serve its entries.
template <uint32_t NT, int D, int KB, bool G, class RM>
__device__ __forceinline__ void level_tile(uint32_t blk, const PairMeta* __restrict__ pm,
                                           const MKey<KB, G>* __restrict__ ent_key, RM rm,
                                           const uint32_t* __restrict__ pos, uint32_t pos_stride,
                                           const uint64_t* __restrict__ res, uint32_t d_rt,
                                           uint16_t* __restrict__ level) {
    constexpr uint32_t E = kPairTileMax / NT;
    const uint32_t ni = pm->n_ins, T = pair_tile(ni + pm->n_del);
    const uint32_t lo = blk * T;
    if (lo >= ni) return;
    const uint32_t hi = min(ni, lo + T), d = D ? uint32_t(D) : d_rt;
    bool in[E];  // an insert entry of an owner-computed sketch (its pairs hold its snapshots)
    // Every load below is unconditional, at an index that always exists (the
    // tile's first entry, pair 0) where the entry is not one of these, so
    // that all of a loop's loads are in flight together; the values loaded
    // for such slots are never used.
#pragma unroll
    for (uint32_t j = 0; j < E; j++) {
        const uint32_t e = lo + j * NT + threadIdx.x;
        const MKey<KB, G> m = ent_key[e < hi ? e : lo];
        in[j] = (e < hi) & rm.has(mkey_sketch<KB, G>(m));
    }
    uint32_t m0[E], dl[E], bm[E];
#pragma unroll
    for (uint32_t j = 0; j < E; j++) m0[j] = dl[j] = bm[j] = kSlimMax;
    for (uint32_t i = 0; i < d; i++) {  // d is a constant when D is
        uint32_t ps[E];
#pragma unroll
        for (uint32_t j = 0; j < E; j++) {
            const uint32_t e = lo + j * NT + threadIdx.x;
            ps[j] = pos[size_t(i) * pos_stride + (in[j] ? e : lo)];
        }
#pragma unroll
        for (uint32_t j = 0; j < E; j++) {
            const uint64_t r = res[in[j] ? ps[j] : 0u];
            m0[j] = min(m0[j], uint32_t(r) & 0xffffu);
            dl[j] = min(dl[j], uint32_t(r >> 16) & 0xffffu);
            bm[j] = min(bm[j], uint32_t(r >> 32) & 0xffffu);
        }
    }
#pragma unroll
    for (uint32_t j = 0; j < E; j++) {
        const uint32_t e = lo + j * NT + threadIdx.x;
        if (!in[j]) continue;
        const uint32_t rise = m0[j] + dl[j], lvl = max(m0[j], bm[j]);
        level[e] = uint16_t(min(min(rise, lvl), kSlimMax));
    }
}

template <int D, int KB, bool G, class RM>
__global__ __launch_bounds__(kPairThreads) void k_level(const PairMeta* __restrict__ pm,
                                                        const MKey<KB, G>* __restrict__ ent_key, RM rm,
                                                        const uint32_t* __restrict__ pos, uint32_t pos_stride,
                                                        const uint64_t* __restrict__ res, uint32_t d_rt,
                                                        uint16_t* __restrict__ level) {
    level_tile<kPairThreads, D, KB, G, RM>(blockIdx.x, pm, ent_key, rm, pos, pos_stride, res, d_rt, level);
}

// A lone sketch on one stream: k_level of batch k and k_part_count of batch
// k + 1 in one launch (the first count_tiles workgroups count, the others
// take level tiles).  Neither reads what the other writes, and both are too
// short to fill the GPU alone.
template <int KB, class P, uint32_t OPS, int D>
__global__ __launch_bounds__(kPartThreads) void k_part_count_level(P plan, uint32_t* __restrict__ hist_out,
                                                                   uint32_t nb_log2, uint32_t count_tiles,
                                                                   const PairMeta* __restrict__ pm,
                                                                   const MKey<KB, false>* __restrict__ ent_key,
                                                                   const uint32_t* __restrict__ pos,
                                                                   uint32_t pos_stride,
                                                                   const uint64_t* __restrict__ res, uint32_t d_rt,
                                                                   uint16_t* __restrict__ level) {
    if (blockIdx.x < count_tiles) {
        part_count_tile<KB, false, P, OPS>(plan, hist_out, nb_log2, blockIdx.x, count_tiles);
        return;
    }
    level_tile<kPartThreads, D, KB, false, LoneRanges>(blockIdx.x - count_tiles, pm, ent_key, LoneRanges{}, pos,
                                                       pos_stride, res, d_rt, level);
}

// One owner step of one (row, range), its records staged in LDS (the range's
// Fat buckets and Slim words, (z + 1) << cr_shift words at most): first the
// end of batch k (pairs_f), then the start of batch k + 1 (pairs_i); either
// may be absent.  Nothing else touches these records between the two: the
// partition, merge and pair kernels of batch k + 1 read keys and entries only.
//   batch k:     A = max(A, T) for its insert pairs (S3); B -= count for its
//                delete pairs (S4); then A = min(A, max_k B) on every cell a
//                delete touched (S5; min with the same value is idempotent)
//   batch k + 1: each insert pair's Slim counter and Fat counter before the
//                batch (S1), the counts added (S2), and its counter after it:
//                res[p] = (A, growth, Bpost), each capped at 65535 (T is
//                capped there, so the caps change no T)
// The range is read once and written once per step.
template <class SR, class RM, uint32_t NT = kOwnThreads>
__global__ __launch_bounds__(NT) void k_own_step(SR sr, RM rm, OwnerGeom og,
                                                          const PairMeta* __restrict__ pm_f,
                                                          const uint64_t* __restrict__ pairs_f,
                                                          const uint16_t* __restrict__ level,
                                                          const PairMeta* __restrict__ pm_i,
                                                          const uint64_t* __restrict__ pairs_i,
                                                          uint64_t* __restrict__ res) {
    extern __shared__ uint32_t L[];  // ncells records of rs words
    constexpr uint32_t T = NT;
    constexpr uint32_t K = 4;   // this batch's insert pairs per thread held in registers (more: through res)
    constexpr uint32_t KF = 4;  // the previous batch's insert pairs per thread held in registers (more: a loop)
    constexpr uint32_t KD = 2;  // ... and its delete pairs
    const uint32_t d = og.d;
    uint32_t row, q;
    owner_of(og, d, row, q);
    const uint32_t ci = row * og.R + q, cd = d * og.R + ci;
    const uint32_t fi0 = pm_f ? pm_f->start[ci] : 0u, fi1 = pm_f ? pm_f->start[ci + 1] : 0u;
    const uint32_t fd0 = pm_f ? pm_f->start[cd] : 0u, fd1 = pm_f ? pm_f->start[cd + 1] : 0u;
    const uint32_t i0 = pm_i ? pm_i->start[ci] : 0u, i1 = pm_i ? pm_i->start[ci + 1] : 0u;
    if (fi0 == fi1 && fd0 == fd1 && i0 == i1) return;  // the range's records stay as they are
    uint32_t sk, range;
    rm.range_of(q, sk, range);
    const SketchDesc sd = sr.of(sk);
    const uint32_t z = sd.g.z, rs = sd.g.rs, zmask = (1u << og.zbits) - 1;
    const uint32_t cell0 = range << og.cr_shift;
    const uint32_t ncells = min(1u << og.cr_shift, sd.g.w - cell0);
    const uint32_t nw = ncells * rs;
    uint32_t* rec0 = sd.fat + (size_t(row) * sd.g.w + cell0) * rs;
    auto cell_of = [&](uint64_t pr) { return ((uint32_t(pr >> 32) & 0xffffu) >> og.zbits) * rs; };
    auto slot_of = [&](uint64_t pr) { return uint32_t(pr >> 32) & zmask; };
    // The pairs (and the T of the previous batch's inserts) do not depend on
    // the records: their loads go out first, then the range's, so that all of
    // them are in flight together.  Each load is unconditional inside a
    // uniform branch (a slot past the column's end reloads its last pair and
    // is skipped below): a load guarded per lane would be waited for at once.
    uint64_t qf[KF] = {}, qd[KD] = {}, qi[K] = {};
    if (fi0 != fi1) {
#pragma unroll
        for (uint32_t k = 0; k < KF; k++) qf[k] = pairs_f[min(fi0 + k * T + threadIdx.x, fi1 - 1)];
    }
    if (fd0 != fd1) {
#pragma unroll
        for (uint32_t k = 0; k < KD; k++) qd[k] = pairs_f[min(fd0 + k * T + threadIdx.x, fd1 - 1)];
    }
    if (i0 != i1) {
#pragma unroll
        for (uint32_t k = 0; k < K; k++) qi[k] = pairs_i[min(i0 + k * T + threadIdx.x, i1 - 1)];
    }
    // the range in 16-byte pieces where it is 16-byte aligned: the first U per
    // thread held in registers, the rest (larger ranges) copied by a loop
    constexpr uint32_t U = 6;
    const bool vec = (reinterpret_cast<uintptr_t>(rec0) & 15u) == 0;
    const uint32_t n4 = vec ? nw / 4 : 0u;
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // a native vector: stays in registers
    const v4u* src4 = reinterpret_cast<const v4u*>(rec0);
    v4u sv[U];  // (read only where u * T + threadIdx.x < n4)
    if (n4) {
#pragma unroll
        for (uint32_t u = 0; u < U; u++) sv[u] = src4[min(u * T + threadIdx.x, n4 - 1)];
    }
    uint32_t lv[KF] = {};
    if (fi0 != fi1) {
#pragma unroll
        for (uint32_t k = 0; k < KF; k++) lv[k] = level[uint32_t(qf[k])];
    }
    {
        v4u* dst = reinterpret_cast<v4u*>(L);
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
            if (u * T + threadIdx.x < n4) dst[u * T + threadIdx.x] = sv[u];
        for (uint32_t i = U * T + threadIdx.x; i < n4; i += T) dst[i] = src4[i];
        for (uint32_t i = 4 * n4 + threadIdx.x; i < nw; i += T) L[i] = rec0[i];
    }
    __syncthreads();
    if (fi0 != fi1 || fd0 != fd1) {
#pragma unroll
        for (uint32_t k = 0; k < KF; k++)
            if (fi0 + k * T + threadIdx.x < fi1) atomicMax(&L[cell_of(qf[k]) + z], lv[k]);
        for (uint32_t p = fi0 + KF * T + threadIdx.x; p < fi1; p += T) {
            const uint64_t pr = pairs_f[p];
            atomicMax(&L[cell_of(pr) + z], uint32_t(level[uint32_t(pr)]));
        }
#pragma unroll
        for (uint32_t k = 0; k < KD; k++)
            if (fd0 + k * T + threadIdx.x < fd1) atomicSub(&L[cell_of(qd[k]) + slot_of(qd[k])], uint32_t(qd[k] >> 48));
        for (uint32_t p = fd0 + KD * T + threadIdx.x; p < fd1; p += T) {
            const uint64_t pr = pairs_f[p];
            atomicSub(&L[cell_of(pr) + slot_of(pr)], uint32_t(pr >> 48));
        }
        __syncthreads();
        auto clamp = [&](uint64_t pr) {
            uint32_t* r = L + cell_of(pr);
            uint32_t m = 0;
            for (uint32_t f = 0; f < z; f++) m = max(m, r[f]);
            atomicMin(r + z, m);
        };
#pragma unroll
        for (uint32_t k = 0; k < KD; k++)
            if (fd0 + k * T + threadIdx.x < fd1) clamp(qd[k]);
        for (uint32_t p = fd0 + KD * T + threadIdx.x; p < fd1; p += T) clamp(pairs_f[p]);
        __syncthreads();
    }
    if (i0 != i1) {
        uint32_t pre[K], a[K];
#pragma unroll
        for (uint32_t k = 0; k < K; k++) {
            const bool in = i0 + k * T + threadIdx.x < i1;
            const uint32_t* r = L + cell_of(qi[k]);
            pre[k] = in ? r[slot_of(qi[k])] : 0u;
            a[k] = in ? r[z] : 0u;
        }
        // pairs beyond the registers keep (A, Bpre) in their own res word meanwhile
        for (uint32_t p = i0 + K * T + threadIdx.x; p < i1; p += T) {
            const uint64_t pr = pairs_i[p];
            const uint32_t* r = L + cell_of(pr);
            res[p] = uint64_t(r[z]) | (uint64_t(r[slot_of(pr)]) << 32);
        }
        __syncthreads();  // every snapshot taken before a counter moves
#pragma unroll
        for (uint32_t k = 0; k < K; k++)
            if (i0 + k * T + threadIdx.x < i1) atomicAdd(&L[cell_of(qi[k]) + slot_of(qi[k])], uint32_t(qi[k] >> 48));
        for (uint32_t p = i0 + K * T + threadIdx.x; p < i1; p += T) {
            const uint64_t pr = pairs_i[p];
            atomicAdd(&L[cell_of(pr) + slot_of(pr)], uint32_t(pr >> 48));
        }
        __syncthreads();
        auto pack = [&](uint32_t p, uint64_t pr, uint32_t av, uint32_t bpre) {
            const uint32_t post = L[cell_of(pr) + slot_of(pr)];
            const uint32_t grow = post - bpre;  // uint32, modular like the counter
            res[p] = uint64_t(av) | (uint64_t(grow < kSlimMax ? grow : kSlimMax) << 16) |
                     (uint64_t(post < kSlimMax ? post : kSlimMax) << 32);
        };
#pragma unroll
        for (uint32_t k = 0; k < K; k++) {
            const uint32_t p = i0 + k * T + threadIdx.x;
            if (p < i1) pack(p, qi[k], a[k], pre[k]);
        }
        for (uint32_t p = i0 + K * T + threadIdx.x; p < i1; p += T) {
            const uint64_t sv = res[p];
            pack(p, pairs_i[p], uint32_t(sv), uint32_t(sv >> 32));
        }
        __syncthreads();
    }
    {
        uint4* dst = reinterpret_cast<uint4*>(rec0);
        const uint4* src = reinterpret_cast<const uint4*>(L);
#pragma unroll 4
        for (uint32_t i = threadIdx.x; i < n4; i += T) dst[i] = src[i];
#pragma unroll 4
        for (uint32_t i = 4 * n4 + threadIdx.x; i < nw; i += T) rec0[i] = L[i];
    }
}

}  // namespace sfk
