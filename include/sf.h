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

/* Frees every device buffer of the sketch after its stream drains. */
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

/* Mixed stream of n ops: ops[t] = 0 inserts keys[t], 1 deletes it (device). */
int sf_update(sf_sketch *sk, const void *keys, const uint8_t *ops, uint64_t n);

/* Point query (Section 3.1 query rule, unchanged in SF_F): out[t] = the
 * smallest of the d Slim counters of keys[t], as uint32 (device pointer). */
int sf_query(sf_sketch *sk, const void *keys, uint64_t n, uint32_t *out);

/* Collector-side point query over an exported Slim (slim: device pointer to
 * [d][w] uint16, row-major) without a sketch; runs on hip_stream. */
int sf_query_slim(const uint16_t *slim, const sf_config *cfg, const void *keys, uint64_t n,
                  uint32_t *out, void *hip_stream);

/* Slim export, the structure sent to the collector (Sections 1 and 3): d*w
 * uint16 counters, row-major [d][w].  out may be host or device memory with
 * room for out_elems >= d*w elements.  Synchronous. */
int sf_export_slim(sf_sketch *sk, uint16_t *out, uint64_t out_elems);

/* Fat export: d*w*z uint32 counters, [d][w][z] (row, bucket, slot), host or
 * device memory, out_elems >= d*w*z.  Synchronous. */
int sf_export_fat(sf_sketch *sk, uint32_t *out, uint64_t out_elems);

/* Wait for all work enqueued on the sketch's stream. */
int sf_sync(sf_sketch *sk);

/* Launch shape of the duplicate-merging kernels: each workgroup groups the
 * keys of a tile of tile_ops consecutive ops (256, 1024 or 2048; default
 * 2048) and issues one atomic per distinct key.  Results do not depend on
 * it; throughput on skewed streams does. */
int sf_set_tile(sf_sketch *sk, uint32_t tile_ops);

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
    SF_K_COUNT = 8
};

typedef struct sf_kernel_stats {
    double ms[SF_K_COUNT];
    uint64_t launches[SF_K_COUNT];
    uint64_t items[SF_K_COUNT];
} sf_kernel_stats;

int sf_profile(sf_sketch *sk, int enable);
int sf_profile_read(sf_sketch *sk, sf_kernel_stats *out, int reset);

/* Static text of a status code. */
const char *sf_strerror(int status);

/* Detail of the calling thread's last error ("" if none). */
const char *sf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SF_H */
