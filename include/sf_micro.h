/*
 * sf_micro.h -- measurement kernels of libsf_micro.so (gfx950).
 *
 * Not part of the sketch: they give the ceilings the sketch kernels are
 * compared against.  The sketch's hot loops are random 4-byte reads and
 * device-scope atomics on arrays of 1 MiB .. 256 MiB (Section 3.4 structure:
 * d hashed counters per op), so the relevant ceiling is the random access
 * rate at that footprint, not streaming bandwidth.
 *
 * All pointers are device pointers; all calls are asynchronous on
 * hip_stream and return 0 or a negative sf_status-style code (-1 invalid
 * argument, -3 launch failure).
 */
#ifndef SF_MICRO_H
#define SF_MICRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Streaming copy of `bytes` (multiple of 16, both pointers 16-byte aligned):
 * a kernel of known traffic, used to calibrate hardware byte counters. */
int micro_copy(const void *src, void *dst, uint64_t bytes, void *hip_stream);

/* n random 4-byte loads from table[0 .. elems) (elems a power of two), indices
 * from a counter-based hash of (access number, seed); the XOR of the loaded
 * values goes to sink[0] so the loads are not optimised away. */
int micro_gather_u32(const uint32_t *table, uint64_t elems, uint64_t n, uint32_t seed,
                     uint32_t *sink, void *hip_stream);

/* n random device-scope relaxed atomic adds of 1 into table[0 .. elems). */
int micro_atomic_add_u32(uint32_t *table, uint64_t elems, uint64_t n, uint32_t seed,
                         void *hip_stream);

/* n random relaxed atomic adds of 1 where each workgroup only touches the
 * 1/nxcc slice of the table that belongs to the XCD it runs on (read from the
 * XCC_ID hardware register); wg_scope != 0 uses workgroup-scope atomics.
 * nxcc and elems are powers of two, elems >= 64 * nxcc. */
int micro_atomic_add_xcd(uint32_t *table, uint64_t elems, uint64_t n, uint32_t seed, uint32_t nxcc,
                         uint32_t wg_scope, void *hip_stream);

/* n accesses of two 4-byte loads each: the second one 64 bytes away in the
 * same aligned 128-byte block (same_line != 0) or at an independent random
 * index.  Tells whether co-locating two counters in one line saves a fetch. */
int micro_gather_pair(const uint32_t *table, uint64_t elems, uint64_t n, uint32_t seed,
                      uint32_t same_line, uint32_t *sink, void *hip_stream);

/* n random 8-byte stores into table[0 .. elems) (elems a power of two,
 * counted in uint64): the rate of writing items out in another order. */
int micro_scatter_u64(uint64_t *table, uint64_t elems, uint64_t n, uint32_t seed, void *hip_stream);

/* XCDs (XCCs) of the current device, or -3 on error. */
int micro_num_xcc(void);

/* n random aligned 16-byte loads (one Fat bucket of four uint32) from
 * table[0 .. elems) (elems a power of two, counted in uint32). */
int micro_gather_16b(const uint32_t *table, uint64_t elems, uint64_t n, uint32_t seed,
                     uint32_t *sink, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SF_MICRO_H */
