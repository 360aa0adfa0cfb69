// Device-side building blocks of the SF-sketch kernels (gfx950, wave64):
// key loads, MurmurHash3 row hashing in registers, the Eq. (1) index split,
// and the LDS tile grouping that merges duplicate keys before they reach a
// counter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfk {

constexpr int kMaxD = 16;
constexpr uint32_t kSlimMax = 65535u;
constexpr int kBlock = 256;  // 4 wavefronts

// Sizes of one sketch's arrays and its index split.
struct Geom {
    uint32_t d, w, z, seed_base;
    uint32_t rs;       // words per cell record: the z Fat counters, then the Slim working copy
    uint32_t pow2;     // w and z are powers of two: masks and shifts
    uint32_t wz32;     // w*z mod 2^32 (0 encodes 2^32)
    uint32_t w_mask;   // w - 1 (pow2 only)
    uint32_t wz_mask;  // w*z - 1 (pow2 only)
    uint32_t w_shift;  // log2(w) (pow2 only)
};

// ---------------------------------------------------------------- keys

template <int KB> struct Key;
template <> struct Key<4> { uint32_t v[1]; };
template <> struct Key<13> { uint32_t v[4]; };  // bytes 0-3, 4-7, 8-11, byte 12

template <int KB> __device__ __forceinline__ Key<KB> load_key(const uint8_t* keys, uint32_t t);

// uint32 keys: one coalesced dword per lane.
template <>
__device__ __forceinline__ Key<4> load_key<4>(const uint8_t* keys, uint32_t t) {
    Key<4> k;
    k.v[0] = reinterpret_cast<const uint32_t*>(keys)[t];
    return k;
}

// 13-byte keys: each lane reads the four aligned dwords that cover its 13
// bytes (neighbouring lanes' windows overlap, so a wavefront reads one
// contiguous span) and funnel-shifts them into place.  Every one of the four
// dwords holds at least one byte of this key, so no load touches a word that
// lies wholly outside the key array.
template <>
__device__ __forceinline__ Key<13> load_key<13>(const uint8_t* keys, uint32_t t) {
    uintptr_t a = reinterpret_cast<uintptr_t>(keys) + 13ull * t;
    const uint32_t* p = reinterpret_cast<const uint32_t*>(a & ~uintptr_t(3));
    uint32_t o = uint32_t(a & 3u);
    uint32_t x0 = p[0], x1 = p[1], x2 = p[2], x3 = p[3];
    Key<13> k;
    k.v[0] = __builtin_amdgcn_alignbyte(x1, x0, o);
    k.v[1] = __builtin_amdgcn_alignbyte(x2, x1, o);
    k.v[2] = __builtin_amdgcn_alignbyte(x3, x2, o);
    k.v[3] = (x3 >> (8u * o)) & 0xffu;
    return k;
}

template <int KB>
__device__ __forceinline__ bool key_eq(const Key<KB>& a, const Key<KB>& b) {
    bool e = true;
#pragma unroll
    for (int j = 0; j < int(sizeof(a.v) / 4); j++) e = e && (a.v[j] == b.v[j]);
    return e;
}

// ---------------------------------------------------------------- hashing
// MurmurHash3_x86_32 split into its seed-independent block mixing (done once
// per key) and the per-seed rounds (done once per row).

__device__ __forceinline__ uint32_t mm_mix(uint32_t k) {
    k *= 0xcc9e2d51u;
    k = __builtin_rotateleft32(k, 15);
    return k * 0x1b873593u;
}
__device__ __forceinline__ uint32_t mm_round(uint32_t h, uint32_t mk) {
    h ^= mk;
    h = __builtin_rotateleft32(h, 13);
    return h * 5u + 0xe6546b64u;
}
__device__ __forceinline__ uint32_t mm_final(uint32_t h, uint32_t len) {
    h ^= len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

template <int KB> struct Mixed;
template <> struct Mixed<4> {
    uint32_t m0;
    __device__ __forceinline__ explicit Mixed(const Key<4>& k) : m0(mm_mix(k.v[0])) {}
    __device__ __forceinline__ uint32_t row(uint32_t seed) const { return mm_final(mm_round(seed, m0), 4u); }
};
template <> struct Mixed<13> {
    uint32_t m0, m1, m2, mt;
    __device__ __forceinline__ explicit Mixed(const Key<13>& k)
        : m0(mm_mix(k.v[0])), m1(mm_mix(k.v[1])), m2(mm_mix(k.v[2])), mt(mm_mix(k.v[3])) {}
    __device__ __forceinline__ uint32_t row(uint32_t seed) const {
        uint32_t h = mm_round(mm_round(mm_round(seed, m0), m1), m2);
        return mm_final(h ^ mt, 13u);
    }
};

// Eq. (1), 0-based: c = g mod wz, bucket h = c mod w, slot f = c div w.
__device__ __forceinline__ void split(const Geom& g, uint32_t hash, uint32_t& h, uint32_t& f) {
    if (g.pow2) {
        uint32_t c = hash & g.wz_mask;
        h = c & g.w_mask;
        f = c >> g.w_shift;
    } else {
        uint32_t c = g.wz32 ? hash % g.wz32 : hash;
        h = c % g.w;
        f = c / g.w;
    }
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

// ---------------------------------------------------------------- tile grouping
// A workgroup takes a tile of kBlock*J consecutive ops and groups its active
// ops by key in an LDS hash table (open addressing, 2x the tile, so probing
// always ends).  Each occupied slot then acts once for all of its ops: one
// Fat atomic carrying the group size, or one Slim raise / clamp.  The owner
// op of a slot (the first to claim it) depends on timing, but every op of a
// key computes the same value, so results do not.
constexpr uint32_t kEmpty = 0xffffffffu;

template <int KB> __device__ __forceinline__ uint32_t slot_hash(const Key<KB>& k) {
    uint32_t h = 0x9e3779b9u;
#pragma unroll
    for (int j = 0; j < int(sizeof(k.v) / 4); j++) h = mm_round(h, mm_mix(k.v[j]));
    return mm_final(h, 0u);
}

template <int KB, int J> struct TileLDS {
    static constexpr uint32_t kOps = uint32_t(kBlock) * J;
    static constexpr uint32_t kSlots = 2 * kOps;
    Key<KB> key[kOps];      // key of each op of the tile (by local index)
    uint32_t owner[kSlots]; // local index of the op that claimed the slot, or kEmpty
    uint32_t cnt[kSlots];   // ops of the slot's key in the tile
};

template <int KB, int J>
__device__ __forceinline__ void tile_clear(TileLDS<KB, J>& L) {
    for (uint32_t s = threadIdx.x; s < TileLDS<KB, J>::kSlots; s += kBlock) {
        L.owner[s] = kEmpty;
        L.cnt[s] = 0;
    }
}

// Insert local op `idx` (key k) into the table; L.key[idx] must already hold k
// for every inserted op (a barrier separates the key stores from the probing).
template <int KB, int J>
__device__ __forceinline__ void tile_insert(TileLDS<KB, J>& L, const Key<KB>& k, uint32_t idx) {
    constexpr uint32_t mask = TileLDS<KB, J>::kSlots - 1;
    uint32_t s = slot_hash<KB>(k) & mask;
    for (uint32_t probe = 0; probe < TileLDS<KB, J>::kSlots; probe++) {
        const uint32_t prev = atomicCAS(&L.owner[s], kEmpty, idx);
        if (prev == kEmpty || key_eq<KB>(L.key[prev], k)) {
            atomicAdd(&L.cnt[s], 1u);
            return;
        }
        s = (s + 1) & mask;
    }
}

__device__ __forceinline__ void atomic_add_u32(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_max_u32(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_min_u32(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace sfk
