// libsf_micro.so: copy and random-access microbenchmarks (see sf_micro.h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sf_micro.h"

namespace {

constexpr int kBlock = 256;
constexpr int kPerThread = 8;  // independent accesses in flight per lane

__device__ __forceinline__ uint32_t mix32(uint32_t x) {  // lowbias32 integer hash
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ uint64_t rand_index(uint64_t a, uint32_t seed, uint64_t mask) {
    uint32_t lo = mix32(uint32_t(a) ^ seed);
    uint32_t hi = mix32(uint32_t(a >> 32) ^ lo ^ 0x9e3779b9u);
    return ((uint64_t(hi) << 32) | lo) & mask;
}

__global__ __launch_bounds__(kBlock) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                 uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kBlock)
        dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void k_gather(const uint32_t* __restrict__ t, uint64_t mask, uint64_t n,
                                                   uint32_t seed, uint32_t* __restrict__ sink) {
    const uint64_t base = (uint64_t(blockIdx.x) * kBlock + threadIdx.x) * kPerThread;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kPerThread; j++) {
        const uint64_t a = base + j;
        if (a < n) acc ^= t[rand_index(a, seed, mask)];
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // practically never; keeps the loads live
}

__global__ __launch_bounds__(kBlock) void k_atomic(uint32_t* __restrict__ t, uint64_t mask, uint64_t n,
                                                   uint32_t seed) {
    const uint64_t base = (uint64_t(blockIdx.x) * kBlock + threadIdx.x) * kPerThread;
#pragma unroll
    for (int j = 0; j < kPerThread; j++) {
        const uint64_t a = base + j;
        if (a < n)
            __hip_atomic_fetch_add(&t[rand_index(a, seed, mask)], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(kBlock) void k_gather16(const uint4* __restrict__ t, uint64_t mask, uint64_t n,
                                                     uint32_t seed, uint32_t* __restrict__ sink) {
    const uint64_t base = (uint64_t(blockIdx.x) * kBlock + threadIdx.x) * kPerThread;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kPerThread; j++) {
        const uint64_t a = base + j;
        if (a < n) {
            const uint4 v = t[rand_index(a, seed, mask)];
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

// Each workgroup reads the XCD (XCC) it runs on from the hardware register and
// only touches that XCD's 1/nxcc slice of the table, so no cache line is
// shared between XCDs.  wg_scope selects workgroup-scope atomics (performed
// in the XCD's own L2) instead of agent scope.
__global__ __launch_bounds__(kBlock) void k_atomic_xcd(uint32_t* __restrict__ t, uint64_t part_mask,
                                                       uint32_t part_shift, uint32_t nxcc, uint64_t n,
                                                       uint32_t seed, uint32_t wg_scope) {
    const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) % nxcc;
    const uint64_t base = (uint64_t(blockIdx.x) * kBlock + threadIdx.x) * kPerThread;
#pragma unroll
    for (int j = 0; j < kPerThread; j++) {
        const uint64_t a = base + j;
        if (a < n) {
            uint32_t* p = &t[(uint64_t(xcc) << part_shift) | rand_index(a, seed, part_mask)];
            if (wg_scope)
                __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
                __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Two 4-byte loads per access: the second 64 bytes away inside the same
// aligned 128-byte block (same_line) or at an independent random index.
__global__ __launch_bounds__(kBlock) void k_gather_pair(const uint32_t* __restrict__ t, uint64_t mask,
                                                        uint64_t n, uint32_t seed, uint32_t same_line,
                                                        uint32_t* __restrict__ sink) {
    const uint64_t base = (uint64_t(blockIdx.x) * kBlock + threadIdx.x) * kPerThread;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kPerThread; j++) {
        const uint64_t a = base + j;
        if (a < n) {
            const uint64_t r = rand_index(a, seed, mask);
            const uint64_t r2 = same_line ? (r ^ 16u) : rand_index(a, seed ^ 0x5bd1e995u, mask);
            acc ^= t[r] + t[r2];
        }
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

// Random 8-byte stores (no read of the old value): the write half of a
// transposition between two orders of the same items.
__global__ __launch_bounds__(kBlock) void k_scatter64(uint64_t* __restrict__ t, uint64_t mask, uint64_t n,
                                                      uint32_t seed) {
    const uint64_t base = (uint64_t(blockIdx.x) * kBlock + threadIdx.x) * kPerThread;
#pragma unroll
    for (int j = 0; j < kPerThread; j++) {
        const uint64_t a = base + j;
        if (a < n) t[rand_index(a, seed, mask)] = a;
    }
}

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

unsigned grid_of(uint64_t n) {
    const uint64_t g = (n + uint64_t(kBlock) * kPerThread - 1) / (uint64_t(kBlock) * kPerThread);
    return unsigned(g);
}

int done() { return hipGetLastError() == hipSuccess ? 0 : -3; }

}  // namespace

extern "C" {

int micro_copy(const void* src, void* dst, uint64_t bytes, void* st) {
    if (!src || !dst || (bytes & 15) || ((uintptr_t(src) | uintptr_t(dst)) & 15)) return -1;
    const uint64_t n = bytes / 16;
    const unsigned grid = unsigned(n / kBlock + 1 < 8192 ? n / kBlock + 1 : 8192);
    k_copy<<<grid, kBlock, 0, static_cast<hipStream_t>(st)>>>(static_cast<const uint4*>(src),
                                                              static_cast<uint4*>(dst), n);
    return done();
}

int micro_gather_u32(const uint32_t* t, uint64_t elems, uint64_t n, uint32_t seed, uint32_t* sink, void* st) {
    if (!t || !sink || !pow2(elems) || n >= (uint64_t(1) << 40)) return -1;
    k_gather<<<grid_of(n), kBlock, 0, static_cast<hipStream_t>(st)>>>(t, elems - 1, n, seed, sink);
    return done();
}

int micro_atomic_add_u32(uint32_t* t, uint64_t elems, uint64_t n, uint32_t seed, void* st) {
    if (!t || !pow2(elems) || n >= (uint64_t(1) << 40)) return -1;
    k_atomic<<<grid_of(n), kBlock, 0, static_cast<hipStream_t>(st)>>>(t, elems - 1, n, seed);
    return done();
}

int micro_gather_16b(const uint32_t* t, uint64_t elems, uint64_t n, uint32_t seed, uint32_t* sink, void* st) {
    if (!t || !sink || !pow2(elems) || elems < 4 || (uintptr_t(t) & 15) || n >= (uint64_t(1) << 40)) return -1;
    k_gather16<<<grid_of(n), kBlock, 0, static_cast<hipStream_t>(st)>>>(reinterpret_cast<const uint4*>(t),
                                                                        elems / 4 - 1, n, seed, sink);
    return done();
}

int micro_atomic_add_xcd(uint32_t* t, uint64_t elems, uint64_t n, uint32_t seed, uint32_t nxcc,
                         uint32_t wg_scope, void* st) {
    if (!t || !pow2(elems) || !pow2(nxcc) || elems < 64ull * nxcc || n >= (uint64_t(1) << 40)) return -1;
    const uint64_t part = elems / nxcc;
    const uint32_t shift = uint32_t(__builtin_ctzll(part));
    k_atomic_xcd<<<grid_of(n), kBlock, 0, static_cast<hipStream_t>(st)>>>(t, part - 1, shift, nxcc, n, seed,
                                                                           wg_scope);
    return done();
}

int micro_gather_pair(const uint32_t* t, uint64_t elems, uint64_t n, uint32_t seed, uint32_t same_line,
                      uint32_t* sink, void* st) {
    if (!t || !sink || !pow2(elems) || elems < 32 || n >= (uint64_t(1) << 40)) return -1;
    k_gather_pair<<<grid_of(n), kBlock, 0, static_cast<hipStream_t>(st)>>>(t, elems - 1, n, seed, same_line,
                                                                           sink);
    return done();
}

int micro_scatter_u64(uint64_t* t, uint64_t elems, uint64_t n, uint32_t seed, void* st) {
    if (!t || !pow2(elems) || n >= (uint64_t(1) << 40)) return -1;
    k_scatter64<<<grid_of(n), kBlock, 0, static_cast<hipStream_t>(st)>>>(t, elems - 1, n, seed);
    return done();
}

int micro_num_xcc(void) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess) return -3;
    return v;
}

}  // extern "C"
