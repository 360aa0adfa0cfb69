// libsf.so: SF-sketch hot path on MI355X (gfx950) behind the C ABI of sf.h.
//
// Device state of one sketch (all in HBM, allocated once by sf_create):
//   fat   uint32 [d][w][z]  Fat-subsketch, bucket-major (Section 3.4 layout):
//                           one bucket = z consecutive counters (z=4: 16 B)
//   slim  uint32 [d][w]     Slim working copy; values stay <= 65535, so the
//                           exported uint16 array is a narrowing copy.  32-bit
//                           cells give native atomic max/min.
//   bpre  uint32 [d][b]     per-batch snapshot of the insert ops' Fat counters
//   asnap uint16 [d][b]     per-batch snapshot of their Slim counters
//   stage uint16 [d][w]     export staging for host destinations
//
// One schedule batch = up to five kernels on the sketch's stream (the
// kernel boundary is the only grid-wide barrier the schedule needs):
//   k_snapshot   S1  insert ops: Slim and Fat counters before the batch
//   k_fat_update S2  insert ops: Fat += group size (one atomic per distinct
//                    key per wavefront)
//   k_raise      S3  insert ops: T = min(m0 + delta, max(m0, Bmin), 65535);
//                    atomic max into the Slim where T exceeds the snapshot
//   k_fat_update S4  delete ops: Fat -= group size
//   k_clamp      S5  delete ops: atomic min of the Slim with the bucket max
// Queries gather d Slim counters per key and take the minimum.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "sf.h"
#include "sf_device.hpp"

using namespace sfk;

// ====================================================================== kernels

__device__ __forceinline__ bool is_delete(const uint8_t* ops, uint32_t t, uint32_t uniform_del) {
    return ops ? ops[t] != 0 : uniform_del != 0;
}

// S1: snapshot of each insert op's Slim and Fat counters (state before the batch).
template <int KB, int D>
__global__ __launch_bounds__(kBlock) void k_snapshot(const uint8_t* __restrict__ keys,
                                                     const uint8_t* __restrict__ ops,
                                                     uint32_t uniform_del, uint32_t cnt, Geom g,
                                                     const uint32_t* __restrict__ fat,
                                                     const uint32_t* __restrict__ slim,
                                                     uint32_t* __restrict__ bpre,
                                                     uint16_t* __restrict__ asnap, uint32_t stride) {
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= cnt || is_delete(ops, t, uniform_del)) return;
    const Mixed<KB> mx(load_key<KB>(keys, t));
    const uint32_t d = D ? uint32_t(D) : g.d;
#pragma unroll
    for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
        if (i < d) {
            uint32_t h, f;
            split(g, mx.row(g.seed_base + i), h, f);
            const size_t cell = size_t(i) * g.w + h;
            asnap[size_t(i) * stride + t] = uint16_t(slim[cell]);
            bpre[size_t(i) * stride + t] = fat[cell * g.z + f];
        }
    }
}

// Loads the tile's active ops (op type == want_del) into the LDS table.
// Returns after a barrier; the table then holds each distinct key once.
template <int KB, int J>
__device__ __forceinline__ void tile_build(TileLDS<KB, J>& L, const uint8_t* __restrict__ keys,
                                           const uint8_t* __restrict__ ops, uint32_t uniform_del,
                                           uint32_t cnt, uint32_t base, bool want_del) {
    tile_clear<KB, J>(L);
    Key<KB> k[J];
    bool act[J];
#pragma unroll
    for (int j = 0; j < J; j++) {
        const uint32_t idx = uint32_t(j) * kBlock + threadIdx.x;
        const uint32_t t = base + idx;
        act[j] = t < cnt && is_delete(ops, t, uniform_del) == want_del;
        if (act[j]) {
            k[j] = load_key<KB>(keys, t);
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
template <int KB, int D, int J>
__global__ __launch_bounds__(kBlock) void k_fat_update(const uint8_t* __restrict__ keys,
                                                       const uint8_t* __restrict__ ops,
                                                       uint32_t uniform_del, uint32_t cnt, Geom g,
                                                       uint32_t* __restrict__ fat, uint32_t want_del) {
    __shared__ TileLDS<KB, J> L;
    const uint32_t base = blockIdx.x * TileLDS<KB, J>::kOps;
    tile_build<KB, J>(L, keys, ops, uniform_del, cnt, base, want_del != 0);
    const uint32_t d = D ? uint32_t(D) : g.d;
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
                split(g, mx.row(g.seed_base + i), h, f);
                atomic_add_u32(&fat[(size_t(i) * g.w + h) * g.z + f], v);
            }
        }
    }
}

// S3: raise the Slim counters of every inserted key to its water level
// T = min(m0 + delta, max(m0, Bmin), 65535), once per distinct key of the tile.
template <int KB, int D, int J>
__global__ __launch_bounds__(kBlock) void k_raise(const uint8_t* __restrict__ keys,
                                                  const uint8_t* __restrict__ ops,
                                                  uint32_t uniform_del, uint32_t cnt, Geom g,
                                                  const uint32_t* __restrict__ fat,
                                                  uint32_t* __restrict__ slim,
                                                  const uint32_t* __restrict__ bpre,
                                                  const uint16_t* __restrict__ asnap, uint32_t stride) {
    constexpr int R = D ? D : kMaxD;
    __shared__ TileLDS<KB, J> L;
    const uint32_t base = blockIdx.x * TileLDS<KB, J>::kOps;
    tile_build<KB, J>(L, keys, ops, uniform_del, cnt, base, false);
    const uint32_t d = D ? uint32_t(D) : g.d;
    for (uint32_t s = threadIdx.x; s < TileLDS<KB, J>::kSlots; s += kBlock) {
        const uint32_t o = L.owner[s];
        if (o == kEmpty) continue;
        const uint32_t t = base + o;  // any op of the key: all share one snapshot
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
                split(g, mx.row(g.seed_base + i), h, f);
                cell[i] = size_t(i) * g.w + h;
                a[i] = asnap[size_t(i) * stride + t];
                const uint32_t post = fat[cell[i] * g.z + f];
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
            if (uint32_t(i) < d && a[i] < T) atomic_max_u32(&slim[cell[i]], T);
    }
}

// Largest counter of a Fat bucket.
__device__ __forceinline__ uint32_t bucket_max(const uint32_t* __restrict__ fat, size_t cell,
                                               const Geom& g) {
    if (g.z == 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(fat + cell * 4);
        return max(max(v.x, v.y), max(v.z, v.w));
    }
    uint32_t m = 0;
    for (uint32_t j = 0; j < g.z; j++) m = max(m, fat[cell * g.z + j]);
    return m;
}

// S5: clamp the Slim counters of every deleted key to their bucket's max,
// once per distinct key of the tile.
template <int KB, int D, int J>
__global__ __launch_bounds__(kBlock) void k_clamp(const uint8_t* __restrict__ keys,
                                                  const uint8_t* __restrict__ ops,
                                                  uint32_t uniform_del, uint32_t cnt, Geom g,
                                                  const uint32_t* __restrict__ fat,
                                                  uint32_t* __restrict__ slim) {
    __shared__ TileLDS<KB, J> L;
    const uint32_t base = blockIdx.x * TileLDS<KB, J>::kOps;
    tile_build<KB, J>(L, keys, ops, uniform_del, cnt, base, true);
    const uint32_t d = D ? uint32_t(D) : g.d;
    for (uint32_t s = threadIdx.x; s < TileLDS<KB, J>::kSlots; s += kBlock) {
        const uint32_t o = L.owner[s];
        if (o == kEmpty) continue;
        const Mixed<KB> mx(L.key[o]);
#pragma unroll
        for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
            if (i < d) {
                uint32_t h, f;
                split(g, mx.row(g.seed_base + i), h, f);
                const size_t cell = size_t(i) * g.w + h;
                const uint32_t m = bucket_max(fat, cell, g);
                if (slim[cell] > m) atomic_min_u32(&slim[cell], m);
            }
        }
    }
}

// Point query: minimum of the d Slim counters of each key.
template <int KB, int D, typename S>
__global__ __launch_bounds__(kBlock) void k_query(const uint8_t* __restrict__ keys, uint32_t n, Geom g,
                                                  const S* __restrict__ slim,
                                                  uint32_t* __restrict__ out) {
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const Mixed<KB> mx(load_key<KB>(keys, t));
    const uint32_t d = D ? uint32_t(D) : g.d;
    uint32_t q = ~0u;
#pragma unroll
    for (uint32_t i = 0; i < uint32_t(D ? D : kMaxD); i++) {
        if (i < d) {
            uint32_t h, f;
            split(g, mx.row(g.seed_base + i), h, f);
            q = min(q, uint32_t(slim[size_t(i) * g.w + h]));
        }
    }
    out[t] = q;
}

// Narrowing copy of the 32-bit Slim working copy into the uint16 export form.
__global__ __launch_bounds__(kBlock) void k_pack16(const uint32_t* __restrict__ in,
                                                   uint16_t* __restrict__ out, size_t n) {
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock)
        out[i] = uint16_t(in[i]);
}

// ====================================================================== host side

struct ProfRec {
    int kind;
    uint64_t items;
    hipEvent_t a, b;
};

struct sf_sketch {
    sf_config cfg;
    Geom g;
    hipStream_t stream;
    int device;
    uint32_t* fat;
    uint32_t* slim;
    uint16_t* stage;
    uint32_t* bpre;
    uint16_t* asnap;
    uint32_t stride;  // snapshot capacity in ops (= batch_ops)
    uint32_t tile_j;  // ops per thread of the grouping kernels (tile = 256 * tile_j ops)
    bool prof;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> spare;
    sf_kernel_stats acc;
};

namespace {

std::mutex g_mu;
std::unordered_set<const sf_sketch*> g_live;
thread_local std::string g_err;

constexpr uint64_t kMaxBatch = 1ull << 30;
constexpr uint32_t kMaxLaunch = 1u << 30;  // ops per kernel launch (uint32 indexing)

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int device_fail(hipError_t e, const char* what) {
    return fail(SF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool live(const sf_sketch* s) {
    std::lock_guard<std::mutex> lk(g_mu);
    return s && g_live.count(s);
}

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

int validate(const sf_config* c) {
    if (!c) return fail(SF_EINVAL, "null config");
    if (c->d < 1 || c->d > uint32_t(kMaxD)) return fail(SF_EINVAL, "d must be in 1..16");
    if (c->w < 1 || c->z < 1) return fail(SF_EINVAL, "w and z must be >= 1");
    if (uint64_t(c->w) * c->z > (1ull << 32)) return fail(SF_EINVAL, "w*z must be <= 2^32");
    if (c->key_bytes != 4 && c->key_bytes != 13) return fail(SF_EINVAL, "key_bytes must be 4 or 13");
    if (c->batch_ops < 1 || c->batch_ops > kMaxBatch) return fail(SF_EINVAL, "batch_ops must be in 1..2^30");
    return SF_OK;
}

uint64_t round256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct Sizes {
    uint64_t fat, slim, stage, bpre, asnap;
    uint64_t total() const { return fat + slim + stage + bpre + asnap; }
};

Sizes sizes_of(const sf_config* c) {
    Sizes s;
    const uint64_t cells = uint64_t(c->d) * c->w;
    s.fat = round256(cells * c->z * 4);
    s.slim = round256(cells * 4);
    s.stage = round256(cells * 2);
    s.bpre = round256(uint64_t(c->d) * c->batch_ops * 4);
    s.asnap = round256(uint64_t(c->d) * c->batch_ops * 2);
    return s;
}

Geom geom_of(const sf_config* c) {
    Geom g{};
    g.d = c->d;
    g.w = c->w;
    g.z = c->z;
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
int check_gpu_ptr(const void* p, uint64_t bytes, const char* what) {
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

bool host_dest(void* p) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return at.type != hipMemoryTypeDevice && !at.isManaged;
}

hipEvent_t take_event(sf_sketch* s) {
    hipEvent_t e = nullptr;
    if (!s->spare.empty()) {
        e = s->spare.back();
        s->spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Brackets one launch with events on the sketch's stream when profiling.
struct Timed {
    sf_sketch* s;
    ProfRec r;
    Timed(sf_sketch* sk, hipStream_t st, int kind, uint64_t items) : s(sk), r{kind, items, nullptr, nullptr} {
        if (!s || !s->prof) return;
        r.a = take_event(s);
        r.b = take_event(s);
        if (r.a) (void)hipEventRecord(r.a, st);
        st_ = st;
    }
    ~Timed() {
        if (!s || !s->prof || !r.a || !r.b) return;
        (void)hipEventRecord(r.b, st_);
        s->recs.push_back(r);
    }
    hipStream_t st_ = nullptr;
};

int drain_profile(sf_sketch* s) {
    hipError_t err = hipSuccess;
    for (auto& r : s->recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && err == hipSuccess) err = e;
        s->acc.ms[r.kind] += ms;
        s->acc.launches[r.kind] += 1;
        s->acc.items[r.kind] += r.items;
        s->spare.push_back(r.a);
        s->spare.push_back(r.b);
    }
    s->recs.clear();
    return err == hipSuccess ? SF_OK : device_fail(err, "profile events");
}

unsigned grid_for(uint64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

// One schedule batch of cnt ops starting at keys/ops.
template <int KB, int D, int J>
void launch_batch_j(sf_sketch* s, const uint8_t* keys, const uint8_t* ops, uint32_t uniform_del,
                    uint32_t cnt, bool ins, bool del) {
    const dim3 grid(grid_for(cnt)), block(kBlock);
    const dim3 tgrid(unsigned((uint64_t(cnt) + TileLDS<KB, J>::kOps - 1) / TileLDS<KB, J>::kOps));
    if (ins) {
        {
            Timed tm(s, s->stream, SF_K_SNAPSHOT, cnt);
            k_snapshot<KB, D><<<grid, block, 0, s->stream>>>(keys, ops, uniform_del, cnt, s->g, s->fat,
                                                              s->slim, s->bpre, s->asnap, s->stride);
        }
        {
            Timed tm(s, s->stream, SF_K_FAT_ADD, cnt);
            k_fat_update<KB, D, J><<<tgrid, block, 0, s->stream>>>(keys, ops, uniform_del, cnt, s->g, s->fat, 0u);
        }
        {
            Timed tm(s, s->stream, SF_K_RAISE, cnt);
            k_raise<KB, D, J><<<tgrid, block, 0, s->stream>>>(keys, ops, uniform_del, cnt, s->g, s->fat,
                                                               s->slim, s->bpre, s->asnap, s->stride);
        }
    }
    if (del) {
        {
            Timed tm(s, s->stream, SF_K_FAT_SUB, cnt);
            k_fat_update<KB, D, J><<<tgrid, block, 0, s->stream>>>(keys, ops, uniform_del, cnt, s->g, s->fat, 1u);
        }
        {
            Timed tm(s, s->stream, SF_K_CLAMP, cnt);
            k_clamp<KB, D, J><<<tgrid, block, 0, s->stream>>>(keys, ops, uniform_del, cnt, s->g, s->fat, s->slim);
        }
    }
}

template <int KB, int D>
void launch_batch(sf_sketch* s, const uint8_t* keys, const uint8_t* ops, uint32_t uniform_del,
                  uint32_t cnt, bool ins, bool del) {
    switch (s->tile_j) {
        case 1: launch_batch_j<KB, D, 1>(s, keys, ops, uniform_del, cnt, ins, del); break;
        case 4: launch_batch_j<KB, D, 4>(s, keys, ops, uniform_del, cnt, ins, del); break;
        default: launch_batch_j<KB, D, 8>(s, keys, ops, uniform_del, cnt, ins, del); break;
    }
}

template <int KB, int D, typename S>
void launch_query(const uint8_t* keys, uint32_t n, const Geom& g, const S* slim, uint32_t* out,
                  hipStream_t st) {
    k_query<KB, D, S><<<dim3(grid_for(n)), dim3(kBlock), 0, st>>>(keys, n, g, slim, out);
}

#define SF_DISPATCH_KD(kb, d, FN, ...)                                                    \
    do {                                                                                  \
        if ((kb) == 4) {                                                                  \
            if ((d) == 4) FN<4, 4>(__VA_ARGS__);                                          \
            else if ((d) == 8) FN<4, 8>(__VA_ARGS__);                                     \
            else FN<4, 0>(__VA_ARGS__);                                                   \
        } else {                                                                          \
            if ((d) == 4) FN<13, 4>(__VA_ARGS__);                                         \
            else if ((d) == 8) FN<13, 8>(__VA_ARGS__);                                    \
            else FN<13, 0>(__VA_ARGS__);                                                  \
        }                                                                                 \
    } while (0)

template <typename S>
void query_dispatch(uint32_t kb, uint32_t d, const uint8_t* keys, uint32_t n, const Geom& g,
                    const S* slim, uint32_t* out, hipStream_t st) {
    if (kb == 4) {
        if (d == 4) launch_query<4, 4, S>(keys, n, g, slim, out, st);
        else if (d == 8) launch_query<4, 8, S>(keys, n, g, slim, out, st);
        else launch_query<4, 0, S>(keys, n, g, slim, out, st);
    } else {
        if (d == 4) launch_query<13, 4, S>(keys, n, g, slim, out, st);
        else if (d == 8) launch_query<13, 8, S>(keys, n, g, slim, out, st);
        else launch_query<13, 0, S>(keys, n, g, slim, out, st);
    }
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
    const uint32_t uniform_del = kind == kDelete ? 1u : 0u;
    for (uint64_t lo = 0; lo < n; lo += b) {
        const uint32_t cnt = uint32_t(n - lo < b ? n - lo : b);
        const uint8_t* kp = k8 + lo * kb;
        const uint8_t* op = kind == kMixed ? ops + lo : nullptr;
        SF_DISPATCH_KD(kb, s->cfg.d, launch_batch, s, kp, op, uniform_del, cnt, kind != kDelete,
                       kind != kInsert);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SF_OK : device_fail(e, "update launch");
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
    hipError_t e = hipGetDevice(&s->device);
    char* base = nullptr;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&base), sz.total());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return e == hipErrorOutOfMemory ? fail(SF_ENOMEM, "hipMalloc: out of device memory")
                                        : device_fail(e, "sf_create");
    }
    s->fat = reinterpret_cast<uint32_t*>(base);
    s->slim = reinterpret_cast<uint32_t*>(base + sz.fat);
    s->stage = reinterpret_cast<uint16_t*>(base + sz.fat + sz.slim);
    s->bpre = reinterpret_cast<uint32_t*>(base + sz.fat + sz.slim + sz.stage);
    s->asnap = reinterpret_cast<uint16_t*>(base + sz.fat + sz.slim + sz.stage + sz.bpre);
    e = hipMemsetAsync(base, 0, sz.fat + sz.slim, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
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
    hipError_t e2 = hipFree(s->fat);
    for (auto& r : s->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto ev : s->spare) (void)hipEventDestroy(ev);
    delete s;
    if (e != hipSuccess) return device_fail(e, "sf_destroy sync");
    if (e2 != hipSuccess) return device_fail(e2, "sf_destroy free");
    return SF_OK;
}

int sf_reset(sf_sketch* s) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    const Sizes sz = sizes_of(&s->cfg);
    hipError_t e = hipMemsetAsync(s->fat, 0, sz.fat + sz.slim, s->stream);
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

static int query_common(sf_sketch* s, const sf_config* c, const Geom& g, const void* slim, bool slim16,
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
        Timed tm(s, st, SF_K_QUERY, cnt);
        if (slim16)
            query_dispatch<uint16_t>(kb, c->d, k8 + lo * kb, cnt, g, static_cast<const uint16_t*>(slim),
                                     out + lo, st);
        else
            query_dispatch<uint32_t>(kb, c->d, k8 + lo * kb, cnt, g, static_cast<const uint32_t*>(slim),
                                     out + lo, st);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SF_OK : device_fail(e, "query launch");
}

int sf_query(sf_sketch* s, const void* keys, uint64_t n, uint32_t* out) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    return query_common(s, &s->cfg, s->g, s->slim, false, keys, n, out, s->stream);
}

int sf_query_slim(const uint16_t* slim, const sf_config* cfg, const void* keys, uint64_t n,
                  uint32_t* out, void* hip_stream) {
    sf_config c = cfg ? *cfg : sf_config{};
    if (cfg) c.batch_ops = 1;  // not used by queries
    int rc = validate(cfg ? &c : nullptr);
    if (rc) return rc;
    if (n && (rc = check_gpu_ptr(slim, uint64_t(c.d) * c.w * 2, "slim"))) return rc;
    return query_common(nullptr, &c, geom_of(&c), slim, true, keys, n, out, static_cast<hipStream_t>(hip_stream));
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
    uint16_t* dst = host ? s->stage : out;
    const unsigned grid = grid_for(cells) < 4096u ? grid_for(cells) : 4096u;
    {
        Timed tm(s, s->stream, SF_K_EXPORT, cells);
        k_pack16<<<dim3(grid), dim3(kBlock), 0, s->stream>>>(s->slim, dst, cells);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && host) e = hipMemcpyAsync(out, s->stage, cells * 2, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_export_slim");
}

int sf_export_fat(sf_sketch* s, uint32_t* out, uint64_t out_elems) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    const uint64_t n = uint64_t(s->cfg.d) * s->cfg.w * s->cfg.z;
    if (!out) return fail(SF_EINVAL, "out is null");
    if (out_elems < n) return fail(SF_EINVAL, "out_elems < d*w*z");
    if (!host_dest(out)) {
        int rc = check_gpu_ptr(out, n * 4, "out");
        if (rc) return rc;
    }
    hipError_t e = hipMemcpyAsync(out, s->fat, n * 4, hipMemcpyDefault, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_export_fat");
}

int sf_sync(sf_sketch* s) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    hipError_t e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? SF_OK : device_fail(e, "sf_sync");
}

int sf_set_tile(sf_sketch* s, uint32_t tile_ops) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    if (tile_ops != 256 && tile_ops != 1024 && tile_ops != 2048)
        return fail(SF_EINVAL, "tile_ops must be 256, 1024 or 2048");
    s->tile_j = tile_ops / kBlock;
    return SF_OK;
}

int sf_profile(sf_sketch* s, int enable) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    s->prof = enable != 0;
    return SF_OK;
}

int sf_profile_read(sf_sketch* s, sf_kernel_stats* out, int reset) {
    if (!live(s)) return fail(SF_ESTATE, "sketch handle is not live");
    int rc = drain_profile(s);
    if (out) *out = s->acc;
    if (reset) s->acc = sf_kernel_stats{};
    return rc;
}

const char* sf_strerror(int status) {
    switch (status) {
        case SF_OK: return "ok";
        case SF_EINVAL: return "invalid argument";
        case SF_ENOMEM: return "out of memory or over the HBM budget";
        case SF_EDEVICE: return "HIP device error";
        case SF_ESTATE: return "sketch handle is not live";
        case SF_EUNDERFLOW: return "delete of an absent item (strict-turnstile violation)";
        default: return "unknown status";
    }
}

const char* sf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
