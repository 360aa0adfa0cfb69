/*
 * sf.h -- C ABI of the MI355X (gfx950) SF-sketch library, libsf.so.
 *
 * The SF-sketch (Yang et al., arXiv:1701.04148) keeps two sets of d hashed
 * arrays: a small Slim-subsketch A (w counters per row) that is shipped to a
 * remote collector and answers queries, and a larger Fat-subsketch B (w
 * buckets of z counters per row) that stays with the monitor and guides the
 * Slim updates (Section 1; structure of Section 3.4, operations of the final
 * version SF_F in Section 3.5).  This library keeps both on one GPU and runs
 * insertions, deletions and point queries over batches of device-resident keys
 * with hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 *  - Return value: SF_OK (0) or a negative sf_status.  Nothing throws across
 *    the ABI.  sf_last_error() gives a detail string for the calling thread.
 *  - Keys are packed, key_bytes bytes each: key_bytes = 4 means uint32 keys
 *    hashed as their 4 little-endian bytes (pointer 4-byte aligned);
 *    key_bytes = 13 means packed 13-byte strings (e.g. 5-tuple flow ids),
 *    stride 13, no alignment requirement.
 *  - Key, op and output pointers passed to update and query calls are DEVICE
 *    pointers owned by the caller; they must stay valid until the work
 *    enqueued on the sketch's stream has completed (sf_sync or a stream
 *    synchronisation).  Update and query calls are asynchronous.
 *  - A sketch is used by one host thread at a time.
 *
 * Hash contract (the paper fixes only "uniform independent hashes", Sections
 * 3.1 and 3.4): row i in [0,d) uses g_i = MurmurHash3_x86_32(key bytes,
 * seed_base + i); the bucket (= Slim column) and slot follow Eq. (1) of
 * Section 3.3 read with 0-based indices: c = g_i mod (w*z), h_i = c mod w,
 * f_i = c div w.
 *
 * Counter widths (not fixed by the paper): Fat counters are uint32 and wrap
 * modulo 2^32; Slim counters are uint16 in every exported form and saturate
 * at 65535, so a query answer of 65535 reads "at least 65535".
 *
 * Update schedule.  SF_F's Slim update depends on op order.  Updates are cut
 * into consecutive batches of cfg.batch_ops ops (every update call starts a
 * new batch); each batch applies, in this order: snapshot of the insert ops'
 * Slim minimum and Fat counters; all Fat increments; the Slim raise of every
 * inserted key to min(m0 + delta, max(m0, Bmin)) (delta = smallest growth of
 * its Fat counters during the batch, Bmin = smallest Fat counter after it,
 * m0 = its smallest Slim counter before it; capped at 65535); all Fat
 * decrements; the Slim clamp A_i[h_i] = min(A_i[h_i], max_k B_i[h_i][k]) of
 * every deleted key.  batch_ops = 1 is exactly the sequential SF_F of
 * Section 3.5.  The result is a pure function of the op sequence and
 * batch_ops: it does not depend on launch shapes or thread timing.
 */
#ifndef SF_H
#define SF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sf_sketch sf_sketch; /* opaque, owned by the library */

typedef struct sf_config {
    uint32_t d;         /* rows of both subsketches, 1..16 */
    uint32_t w;         /* Slim counters per row = Fat buckets per row, >= 1 */
    uint32_t z;         /* Fat counters per bucket, >= 1; w*z <= 2^32 */
    uint32_t key_bytes; /* 4 or 13 */
    uint32_t seed_base; /* row i hashes with seed seed_base + i */
    uint32_t batch_ops; /* ops per schedule batch, >= 1 (1 = sequential SF_F) */
} sf_config;

typedef enum sf_status {
    SF_OK = 0,
    SF_EINVAL = -1,     /* bad config, null or misaligned pointer, size too small */
    SF_ENOMEM = -2,     /* over the HBM budget, or a device allocation failed */
    SF_EDEVICE = -3,    /* a HIP call failed; detail in sf_last_error() */
    SF_ESTATE = -4,     /* handle not live (destroyed or never created) */
    SF_EUNDERFLOW = -5  /* reserved for checked deletes (the oracle); not raised here */
} sf_status;

/* Device bytes sf_create allocates for cfg (Fat, Slim working copy, export
 * staging, per-batch snapshot).  0 if cfg is invalid. */
uint64_t sf_footprint(const sf_config *cfg);

/* Initialisation (Section 3.1: every counter zero).  Validates cfg, checks
 * sf_footprint(cfg) against hbm_budget_bytes (0 = no limit) BEFORE any device
 * call, allocates on the current HIP device, zeroes, and binds the sketch to
 * hip_stream (a hipStream_t; NULL = the null stream).  Blocks until zeroed.
 * Errors: SF_EINVAL, SF_ENOMEM, SF_EDEVICE.  *out is set only on SF_OK. */
int sf_create(const sf_config *cfg, uint64_t hbm_budget_bytes, void *hip_stream, sf_sketch **out);

/* Frees every device buffer of the sketch after its stream drains (the
 * sketch's lifetime; the paper has no counterpart).  SF_ESTATE for a handle
 * that is not live; the handle is dead after the call. */
int sf_destroy(sf_sketch *sk);

/* Re-zero both subsketches (asynchronous on the sketch's stream). */
int sf_reset(sf_sketch *sk);

/* Rebind the sketch to another stream (synchronises the old one first). */
int sf_set_stream(sf_sketch *sk, void *hip_stream);

/* Insertion of n keys (Section 3.4 insertion, used unchanged by SF_F). */
int sf_insert(sf_sketch *sk, const void *keys, uint64_t n);

/* Deletion of n keys (SF_F deletion, Section 3.5).  Precondition (strict
 * turnstile, assumed by the no-under-estimation proof of Appendix II): each
 * deleted key is currently present at least as often as it is deleted.  A
 * violation is not detected: Fat counters wrap, Slim results are undefined. */
int sf_delete(sf_sketch *sk, const void *keys, uint64_t n);

/* Mixed stream of n ops (items inserted and deleted, Section 3; SF_F's
 * insertion of Section 3.4 and deletion of Section 3.5): ops[t] = 0 inserts
 * keys[t], 1 deletes it; keys and ops are device buffers of n entries.  The
 * ops are cut into schedule batches in order; inside a batch inserts apply
 * before deletes (the update schedule above).  Same precondition on deletes
 * as sf_delete.  SF_EINVAL for bad pointers or op buffers shorter than n. */
int sf_update(sf_sketch *sk, const void *keys, const uint8_t *ops, uint64_t n);

/* Host-fed updates: n ops whose keys (and op codes, or NULL for all
 * inserts) are in PINNED host memory (hipHostMalloc).  They are copied in
 * chunks of chunk_ops ops (a positive multiple of batch_ops, so the batches
 * are exactly those of one sf_update call on device buffers) into two device
 * buffers the sketch keeps, on a copy stream of its own: the copy of chunk
 * c+1 overlaps the updates of chunk c.  Returns once every copy from the
 * host buffers has completed (the caller may reuse them); the updates may
 * still run on the sketch's stream.  SF_EINVAL for pageable host memory or a
 * bad chunk size. */
int sf_update_host(sf_sketch *sk, const void *host_keys, const uint8_t *host_ops, uint64_t n,
                   uint64_t chunk_ops);

/* Point query (Section 3.1 query rule, unchanged in SF_F): out[t] = the
 * smallest of the d Slim counters of keys[t], as uint32 (device pointer).
 * Between an sf_export_slim and the next update or reset, the query reads
 * the dense uint16 copy that export made (same values, a fifth of the
 * memory footprint); otherwise it reads the Slim words of the sketch.  A
 * dense copy larger than 4 MiB with d dividing 8 is read one row per XCD:
 * per-row counters go to the sketch's export staging buffer (like every
 * call, ordered on the sketch's stream), then a second pass takes the
 * minimum. */
int sf_query(sf_sketch *sk, const void *keys, uint64_t n, uint32_t *out);

/* Host-fed batched point query, the multi-stream pipeline of the paper's GPU
 * implementation (Section 4.2): n keys in PINNED host memory are split over
 * `streams` HIP streams (1..16) of the sketch's own -- the first n mod streams
 * streams take one key more -- and each stream copies its keys in, runs the
 * query kernel (one pass over the Slim, as sf_query) and copies its answers
 * to host_out (PINNED, n uint32), so the copies of one stream overlap the
 * kernels of another.  The streams start after the work already on the
 * sketch's stream, and later work on that stream waits for them.  Device
 * buffers (one per stream) are allocated on first use and grown when a
 * larger share arrives.  Blocks until every answer is in host_out.  SF_EINVAL
 * for pageable memory or a bad stream count. */
int sf_query_host(sf_sketch *sk, const void *host_keys, uint64_t n, uint32_t *host_out, uint32_t streams);

/* Collector-side point query (Section 3.1 query rule) over an exported Slim
 * (Sections 1 and 3: the collector holds only the Slim): slim is a device
 * pointer to [d][w] uint16, row-major; keys and out as in sf_query; runs on
 * hip_stream (NULL = the null stream).  cfg.batch_ops is ignored.  A Slim
 * larger than 4 MiB with d dividing 8 is read one row per XCD, as sf_query
 * does after an export: per-row counters of runs of keys go to scratch the
 * call allocates stream-ordered (hipMallocAsync / hipFreeAsync on
 * hip_stream); smaller Slims take one pass with no scratch.  Errors:
 * SF_EINVAL (bad config or pointers, buffers too small), SF_ENOMEM (no
 * scratch), SF_EDEVICE. */
int sf_query_slim(const uint16_t *slim, const sf_config *cfg, const void *keys, uint64_t n,
                  uint32_t *out, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): sf_query_slim
 * with the same kernels and the same answers, but the per-row counters live
 * in a static device array of SF_NOALLOC_QUERY_COUNTERS uint16 (16 MiB) that
 * every GPU the library runs on holds until the process ends; the call makes
 * no allocation of any kind.  Limit: n * d <= SF_NOALLOC_QUERY_COUNTERS
 * (e.g. 2M keys at d = 4), whichever path the Slim takes; larger n is
 * rejected with SF_EINVAL before any device work -- split the keys over
 * several calls.  All calls on one GPU share the array: calls that overlap
 * on one GPU (two streams, or two host threads) race and may return wrong
 * answers; calls ordered on one stream are safe.  Other errors as
 * sf_query_slim. */
#define SF_NOALLOC_QUERY_COUNTERS (1u << 23)
int sf_query_slim_noalloc(const uint16_t *slim, const sf_config *cfg, const void *keys, uint64_t n,
                          uint32_t *out, void *hip_stream);

/* Slim export, the structure sent to the collector (Sections 1 and 3): d*w
 * uint16 counters, row-major [d][w].  out may be host or device memory with
 * room for out_elems >= d*w elements.  A host destination is complete when
 * the call returns; a device destination is written in order on the
 * sketch's stream (work later on that stream sees it; another stream must
 * synchronise first, e.g. with sf_sync).  The sketch keeps its own copy of
 * what it exported, for sf_query. */
int sf_export_slim(sf_sketch *sk, uint16_t *out, uint64_t out_elems);

/* Fat export, the Fat-subsketch of Section 3.4's structure (d arrays of w
 * buckets of z counters; Eq. (1) of Section 3.3 gives the bucket and slot):
 * d*w*z uint32 counters, [d][w][z] (row, bucket, slot), to host or device
 * memory, out_elems >= d*w*z.  Synchronous.  It stays with the monitor (the
 * collector gets only the Slim); tests and tools read it.  SF_EINVAL for a
 * null or short destination. */
int sf_export_fat(sf_sketch *sk, uint32_t *out, uint64_t out_elems);

/* Wait for all work enqueued on the sketch's stream (host synchronisation;
 * the paper has no counterpart).  SF_EDEVICE if a kernel failed. */
int sf_sync(sf_sketch *sk);

/* Launch shape of the per-tile merging path (sf_set_merge(sk, 0)): each
 * workgroup groups the keys of a tile of tile_ops consecutive ops (256, 1024
 * or 2048; default 2048) and issues one atomic per distinct key.  Results do
 * not depend on it; throughput on skewed streams does.  The batch-wide path
 * ignores it. */
int sf_set_tile(sf_sketch *sk, uint32_t tile_ops);

/* Where duplicate keys are merged before they reach a counter, and how the
 * merged keys reach the counters.  Modes 1 (the default), 2 and 3 merge
 * across the whole batch: keys are first partitioned into hash buckets, then
 * merged per chunk of whole buckets (a large bucket spans several chunks),
 * and S1..S5 run once per merged key.  Where the shape allows it (a range of
 * 2^k >= 16 cells, at most 1024 ranges per row and at most 8192 / d, holds at
 * most 8192 Fat counters), S1..S5 can run owner-computes: each (row, cell
 * range) has one owning workgroup per step that stages the range's records
 * in LDS and applies S1..S5 there; mode 1 does so for batches of at least w
 * ops and mode 3 for every batch.  Otherwise (smaller batches in mode 1, mode
 * 2, shapes that do not fit) one device-scope atomic per merged key and row
 * applies them.  0 merges per tile of consecutive ops.  Results are identical
 * in every mode (Section 3.4 insertion and Section 3.5 deletion are sums,
 * maxima and minima per counter).  The owner path's buffers (the pairs of two
 * batches, their positions and snapshots: about 28 * d + 2 bytes per op of
 * batch_ops, counted in sf_footprint) are a separate allocation made by
 * sf_create: modes 0 and 2 free it (after the stream drains), modes 1 and 3
 * allocate it again (SF_ENOMEM if they cannot).  SF_EINVAL for other values. */
int sf_set_merge(sf_sketch *sk, int batch_wide);

/* The mode sf_update runs in now: 0 per-tile merging, 1 batch-wide merge with
 * owner-computes S1..S5 for batches of at least w ops, 2 batch-wide merge with
 * atomic S1..S5, 3 owner-computes for every batch; negative on error.  Mode 1
 * or 3 reads 2 when the shape does not fit the owner path. */
int sf_merge_path(sf_sketch *sk);

/* Range size of the owner path: ranges of 2^shift cells per row.  shift 0
 * restores the default (about 512 ranges per row but at least 256 cells,
 * within the allowed sizes: 2048 cells at w = 2^20, 256 at w = 2^14).
 * Ranges of more than 24 KiB of records get 512-thread workgroups, smaller
 * ones 256.  Allowed shifts run from the smallest that keeps a row within
 * min(1024, 8192 / d) ranges (at least 4) to the largest whose range holds
 * at most 8192 Fat counters and 2^16 (cell, slot) codes; SF_EINVAL outside
 * them or when the shape has no owner path.  Takes effect at the next update
 * call; the results do not depend on it. */
int sf_set_owner_range(sf_sketch *sk, uint32_t shift);
/* The current range shift of the owner path; 0 when the shape has none. */
int sf_owner_range(sf_sketch *sk);

/* Streams of the owner path.  With 1 the partition, merge and pair kernels of
 * batch k + 1 run on a second stream of the sketch's (created with the owner
 * buffers, default priority) while the owner steps of batch k run on its own
 * stream; events order the two, and every update call returns with all of
 * its work ordered on the sketch's stream, as with 0 (one stream).  -1 (the
 * default) takes 1 when the cell records (d * w * (z + 1) * 4 bytes) exceed
 * 256 MiB, the Infinity Cache, and 0 otherwise.  Results are the same either
 * way.  SF_EINVAL for other values. */
int sf_set_streams(sf_sketch *sk, int mode);

/* Merged entries (distinct keys per merge chunk) the batch-wide merge has
 * emitted since sf_create, for inserts and deletes; waits for the stream. */
int sf_merge_stats(sf_sketch *sk, uint64_t *insert_entries, uint64_t *delete_entries);

/* ---- per-kernel timing (measurement aid; off by default) ----------------
 * When enabled, every kernel the sketch launches is bracketed by two HIP
 * events recorded on the sketch's stream.  sf_profile_read waits for them
 * and returns, per kernel kind, the summed duration, the launch count and
 * the items (ops, keys or cells) the launches covered; reset != 0 clears
 * the accumulators. */
enum sf_kernel_kind {
    SF_K_SNAPSHOT = 0, /* S1 */
    SF_K_FAT_ADD = 1,  /* S2 */
    SF_K_RAISE = 2,    /* S3 */
    SF_K_FAT_SUB = 3,  /* S4 */
    SF_K_CLAMP = 4,    /* S5 */
    SF_K_QUERY = 5,
    SF_K_EXPORT = 6,
    SF_K_MERGE = 7,    /* batch-wide merge: merge per chunk of bucketed keys */
    SF_K_PARTITION = 8,/* batch-wide merge: bucket counts, starts, scatter */
    SF_K_PAIRS = 9,    /* owner path: (entry, row) pairs partitioned by (row, cell range) */
    SF_K_OWN_STEP = 10,/* owner path: per (row, cell range), S3..S5 of the previous batch, S1 + S2 of this one */
    SF_K_LEVEL = 11,   /* owner path: S3's level T per inserted key */
    SF_K_OWN_FINAL = 12,  /* owner path: S3..S5 of an update call's last batch */
    SF_K_COUNT = 16
};

typedef struct sf_kernel_stats {
    double ms[SF_K_COUNT];
    uint64_t launches[SF_K_COUNT];
    uint64_t items[SF_K_COUNT];
} sf_kernel_stats;

int sf_profile(sf_sketch *sk, int enable);
int sf_profile_read(sf_sketch *sk, sf_kernel_stats *out, int reset);

/* ---- sketch groups -----------------------------------------------------
 * Many independent sketches (e.g. one per monitoring node, Section 1) kept
 * in one allocation and updated by the same launches.  cfgs[i] gives sketch
 * i's shape and schedule (d, w, z, seed_base and batch_ops may differ;
 * key_bytes must be equal).  Every sketch cuts ITS OWN ops into batches of
 * its own batch_ops, so its state is exactly what sf_create + sf_update on
 * the same ops would give.  Round k runs batch k of every sketch;
 * round_ops (0 = min(sum of batch_ops, 2^26), at least the largest
 * batch_ops) bounds the ops one launch covers and sizes the snapshot
 * scratch.  Update calls are recorded into a hipGraph and replayed when the
 * next call has the same segments, buffers and op kind (sf_group_set_graph
 * turns this off).  If hip_stream is NULL the group creates its own
 * (blocking) stream, because graphs cannot be captured on the null stream.
 *
 * Keys of an update or query call are the concatenation of every sketch's
 * keys, sketch 0 first; seg is a HOST array of n+1 offsets (seg[0] = 0,
 * non-decreasing, seg[n] = total keys): sketch i owns keys [seg[i], seg[i+1]).
 * Query answers go to out in the same order. */
typedef struct sf_group sf_group;

uint64_t sf_group_footprint(uint32_t n, const sf_config *cfgs, uint64_t round_ops);
int sf_group_create(uint32_t n, const sf_config *cfgs, uint64_t round_ops, uint64_t hbm_budget_bytes,
                    void *hip_stream, sf_group **out);
int sf_group_destroy(sf_group *g);
int sf_group_reset(sf_group *g);
int sf_group_insert(sf_group *g, const void *keys, const uint64_t *seg);
int sf_group_delete(sf_group *g, const void *keys, const uint64_t *seg);
int sf_group_update(sf_group *g, const void *keys, const uint8_t *ops, const uint64_t *seg);
int sf_group_query(sf_group *g, const void *keys, const uint64_t *seg, uint32_t *out);
int sf_group_export_slim(sf_group *g, uint32_t i, uint16_t *out, uint64_t out_elems);
int sf_group_export_fat(sf_group *g, uint32_t i, uint32_t *out, uint64_t out_elems);
int sf_group_sync(sf_group *g);
int sf_group_set_graph(sf_group *g, int enable);
int sf_group_set_tile(sf_group *g, uint32_t tile_ops);
/* Merge path of the group (default 1): 0 per-tile merging; 1 batch-wide
 * merging with owner-computes S1..S5 when every sketch has the same d and z
 * (ranges of 2^k cells, k the largest with at most 8192 Fat counters and a
 * 16-bit local code per range; a sub-round then also holds at most
 * min(1024, 8192 / d) ranges per row, and no sketch may have more), else as
 * 2; 2 batch-wide merging with atomic S1..S5.
 * Batch-wide merging treats each (key, sketch) pair as one key; merged
 * sub-rounds hold at most 2^24 ops (or the largest batch_ops), tiles of the
 * per-tile path at most round_ops.  The owner-path buffers (counted by
 * sf_group_footprint) are allocated at create time for shapes that qualify,
 * freed by modes 0 and 2 and allocated again by mode 1 (SF_ENOMEM if that
 * fails; the group then runs as mode 2).  SF_EINVAL for another mode.  Waits
 * for the stream; the next update call re-plans. */
int sf_group_set_merge(sf_group *g, int mode);
/* Mode 1 per sketch and round: a sketch's batch takes the owner path when it
 * has at least ratio * w ops, else the atomic entry kernels (both run in
 * one sub-round, each on its own sketches).  The owner path streams all of a
 * sketch's ranges, so a batch that touches them sparsely costs less with
 * atomics.  0 (the default) sends every batch to the owner path.  Results
 * are the same for every ratio.  SF_EINVAL outside [0, 1e6]; waits for the
 * stream; the next update call re-plans. */
int sf_group_set_owner_ratio(sf_group *g, double ratio);
/* The path the next update call takes: 0, 1 or 2 as in sf_group_set_merge. */
int sf_group_merge_path(sf_group *g);
/* As sf_merge_stats, summed over the group's sketches. */
int sf_group_merge_stats(sf_group *g, uint64_t *insert_entries, uint64_t *delete_entries);
/* Sub-rounds (launch groups) and tiles of the last update call's plan. */
int sf_group_rounds(sf_group *g, uint64_t *subrounds, uint64_t *tiles);
int sf_group_profile(sf_group *g, int enable);
int sf_group_profile_read(sf_group *g, sf_kernel_stats *out, int reset);



/* ---- sketch pools: the device side of a serving loop -------------------
 * A pool holds sketches of ONE shape (cfg) in slots of one allocation.  The
 * number of slots is max_slots, or what hbm_budget_bytes holds after the
 * shared buffers (snapshot scratch for round_ops ops -- 0 = 2^24, at least
 * batch_ops -- export staging and an in-flight descriptor ring); both given:
 * the smaller.  A monitoring node's stream acquires a slot when admitted
 * (the slot is zeroed: Section 3.1 initialisation) and releases it when it
 * closes.  sf_pool_launch runs requests of many slots together, AT MOST ONE
 * PER SLOT: each update request is cut into batch_ops batches exactly like
 * one sf_insert / sf_delete / sf_update call on a lone sketch (its own batch
 * boundaries), so a slot ends in the same state alone or in any mix; query
 * requests see their slot after every earlier launch.  Launches run in order
 * on the pool's stream (NULL: the pool creates a blocking stream) and return
 * a ticket; sf_pool_done / sf_pool_wait report completion.  Request buffers
 * must stay valid until their ticket is done. */
typedef struct sf_pool sf_pool;

enum sf_request_kind { SF_REQ_INSERT = 0, SF_REQ_DELETE = 1, SF_REQ_UPDATE = 2, SF_REQ_QUERY = 3 };

typedef struct sf_request {
    const void *keys;   /* device: n keys */
    const uint8_t *ops; /* device: n op codes, 0 insert / 1 delete (SF_REQ_UPDATE only) */
    uint32_t *out;      /* device: n answers (SF_REQ_QUERY only) */
    uint64_t n;
    uint32_t slot;      /* an acquired slot */
    uint32_t kind;      /* sf_request_kind */
} sf_request;

/* Device bytes one slot takes (Fat + Slim working copy + table entry). */
uint64_t sf_pool_slot_bytes(const sf_config *cfg);
int sf_pool_create(const sf_config *cfg, uint32_t max_slots, uint64_t round_ops, uint64_t hbm_budget_bytes,
                   void *hip_stream, sf_pool **out);
int sf_pool_destroy(sf_pool *p);
int sf_pool_capacity(sf_pool *p, uint32_t *slots, uint32_t *free_slots);
/* SF_ENOMEM when every slot is taken (admission control). */
int sf_pool_acquire(sf_pool *p, uint32_t *slot);
int sf_pool_release(sf_pool *p, uint32_t slot);
int sf_pool_launch(sf_pool *p, const sf_request *reqs, uint32_t n, uint64_t *ticket);
/* 1 when the ticket's launch has completed, 0 while pending, < 0 on error. */
int sf_pool_done(sf_pool *p, uint64_t ticket);
int sf_pool_wait(sf_pool *p, uint64_t ticket);
/* Slim of a slot as uint16 [d][w]; async != 0 (device destination only)
 * enqueues the copy on the pool stream without waiting. */
int sf_pool_export_slim(sf_pool *p, uint32_t slot, uint16_t *out, uint64_t out_elems, int async);
int sf_pool_export_fat(sf_pool *p, uint32_t slot, uint32_t *out, uint64_t out_elems);
int sf_pool_sync(sf_pool *p);
int sf_pool_set_tile(sf_pool *p, uint32_t tile_ops);
/* As sf_set_merge for the pool's later launches (default 1); (key, slot)
 * pairs are merged across a sub-round of at most 2^24 ops (or batch_ops).
 * With batch-wide merging, pools whose slots hold at most 64 MiB of records
 * run a request batch of at least ratio * w ops (sf_pool_set_owner_ratio,
 * default 0.5) owner-computes: its slot's (row, range) tiles staged in LDS, a
 * sub-round's owner batches at most 2^22 ops and min(1024, 8192 / d) ranges
 * per row; the other batches of the sub-round take the atomic entry kernels.
 * The owner buffers are part of the shared buffers (fewer slots fit the
 * budget).  Results are the same on either path. */
int sf_pool_set_merge(sf_pool *p, int batch_wide);
/* The owner ratio above; SF_EINVAL for a pool without the owner path or a
 * ratio outside [0, 1e6] (0: every batch that fits the owner buffers). */
int sf_pool_set_owner_ratio(sf_pool *p, double ratio);
/* As sf_merge_stats, summed over all launches of the pool; waits for it. */
int sf_pool_merge_stats(sf_pool *p, uint64_t *insert_entries, uint64_t *delete_entries);

/* Static text of a status code. */
const char *sf_strerror(int status);

/* Detail of the calling thread's last error ("" if none). */
const char *sf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SF_H */
