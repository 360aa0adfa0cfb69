/*
 * SF-sketch CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential C implementation of the Slim-Fat sketch in its
 * final form (SF_F), written from the paper (Yang et al., "SF-sketch: A
 * Two-stage Sketch for Data Streams", arXiv:1701.04148).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never does.  It shares no code with the HIP path: it has
 * its own hash, its own index derivation and its own loops.
 *
 * Structure (Section 3.4, SF_4, reused unchanged by SF_F in Section 3.5):
 *   Slim  A[i][j]      i in [0,d), j in [0,w)              (uint16 here)
 *   Fat   B[i][j][k]   k in [0,z): z counters per bucket    (uint32 here)
 * Row i uses a bucket index h_i(e) in [0,w) and a slot index f_i(e) in [0,z).
 * Initialisation sets every counter to zero (Section 3.1).
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *  - Hash family: MurmurHash3_x86_32 (Appleby, public domain) over the key's
 *    bytes with seed seed_base + i for row i.
 *  - One row hash g_i in [0, 2^32) gives both indices, following Eq. (1) of
 *    Section 3.3 with 0-based indices: c = g mod (w*z), h = c mod w,
 *    f = c div w.
 *  - Counter widths are not fixed by the paper.  Fat counters are uint32
 *    (modular; never exceeded by strict-turnstile streams of < 2^32 ops);
 *    Slim counters are uint16 and saturate at 65535, so a query of 65535
 *    reads "at least 65535".
 *  - Deletion rule of SF_F: "if the bucket max changed, set A to the new max
 *    when A exceeds it" is implemented literally in the sequential mode.
 *
 * Two update modes:
 *  - seq      : strict sequential SF_F, one op at a time (Sections 3.4, 3.5).
 *  - batch(b) : the deterministic batch schedule that the parallel path
 *               reproduces (defined at oracle_batch_idx below).  b = 1 is
 *               the sequential semantics.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_EUNDERFLOW (-5)

#define SLIM_MAX 65535u

typedef struct oracle_sketch {
    uint32_t d, w, z, key_bytes, seed_base;
    uint32_t *B; /* Fat, element (i, j, k) at (i*w + j)*z + k */
    uint16_t *A; /* Slim, element (i, j) at i*w + j */
} oracle_sketch;

/* ------------------------------------------------------------------ hash */

static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

/* MurmurHash3_x86_32 over len bytes, from its published definition. */
uint32_t oracle_murmur3_32(const uint8_t *data, uint64_t len, uint32_t seed)
{
    const uint32_t c1 = 0xcc9e2d51u, c2 = 0x1b873593u;
    uint32_t h = seed;
    uint64_t nblocks = len / 4;
    for (uint64_t b = 0; b < nblocks; b++) {
        const uint8_t *p = data + 4 * b;
        uint32_t k = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) |
                     ((uint32_t)p[3] << 24);
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
        h = rotl32(h, 13);
        h = h * 5u + 0xe6546b64u;
    }
    const uint8_t *tail = data + 4 * nblocks;
    uint32_t k = 0;
    switch (len & 3) {
    case 3:
        k ^= (uint32_t)tail[2] << 16; /* fall through */
    case 2:
        k ^= (uint32_t)tail[1] << 8; /* fall through */
    case 1:
        k ^= (uint32_t)tail[0];
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
    }
    h ^= (uint32_t)len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* Row indices of one key: Eq. (1) read with 0-based indices. */
static void key_indices(const oracle_sketch *s, const uint8_t *key, uint32_t *h, uint32_t *f)
{
    uint64_t wz = (uint64_t)s->w * (uint64_t)s->z;
    for (uint32_t i = 0; i < s->d; i++) {
        uint32_t g = oracle_murmur3_32(key, s->key_bytes, s->seed_base + i);
        uint64_t c = (uint64_t)g % wz;
        h[i] = (uint32_t)(c % s->w);
        f[i] = (uint32_t)(c / s->w);
    }
}

/* ------------------------------------------------------------ lifecycle */

oracle_sketch *oracle_create(uint32_t d, uint32_t w, uint32_t z, uint32_t key_bytes,
                             uint32_t seed_base)
{
    if (d == 0 || w == 0 || z == 0 || key_bytes == 0)
        return NULL;
    if (d > 64)  /* the per-key index buffers of the query and histogram helpers hold 64 rows */
        return NULL;
    if ((uint64_t)w * z > (1ull << 32))
        return NULL;
    oracle_sketch *s = (oracle_sketch *)calloc(1, sizeof(*s));
    if (!s)
        return NULL;
    s->d = d;
    s->w = w;
    s->z = z;
    s->key_bytes = key_bytes;
    s->seed_base = seed_base;
    s->B = (uint32_t *)calloc((size_t)d * w * z, sizeof(uint32_t));
    s->A = (uint16_t *)calloc((size_t)d * w, sizeof(uint16_t));
    if (!s->B || !s->A) {
        free(s->B);
        free(s->A);
        free(s);
        return NULL;
    }
    return s;
}

void oracle_destroy(oracle_sketch *s)
{
    if (!s)
        return;
    free(s->B);
    free(s->A);
    free(s);
}

void oracle_get_state(const oracle_sketch *s, uint32_t *fat, uint16_t *slim)
{
    if (fat)
        memcpy(fat, s->B, (size_t)s->d * s->w * s->z * sizeof(uint32_t));
    if (slim)
        memcpy(slim, s->A, (size_t)s->d * s->w * sizeof(uint16_t));
}

void oracle_set_state(oracle_sketch *s, const uint32_t *fat, const uint16_t *slim)
{
    if (fat)
        memcpy(s->B, fat, (size_t)s->d * s->w * s->z * sizeof(uint32_t));
    if (slim)
        memcpy(s->A, slim, (size_t)s->d * s->w * sizeof(uint16_t));
}

/* Indices of n keys, [n][d] each; lets tests inspect the hash contract. */
void oracle_indices(const oracle_sketch *s, const uint8_t *keys, uint64_t n, uint32_t *h,
                    uint32_t *f)
{
    for (uint64_t t = 0; t < n; t++)
        key_indices(s, keys + t * s->key_bytes, h + t * s->d, f + t * s->d);
}

static uint32_t *fat_at(const oracle_sketch *s, uint32_t i, uint32_t j, uint32_t k)
{
    return &s->B[((uint64_t)i * s->w + j) * s->z + k];
}

static uint16_t *slim_at(const oracle_sketch *s, uint32_t i, uint32_t j)
{
    return &s->A[(uint64_t)i * s->w + j];
}

static uint32_t bucket_max(const oracle_sketch *s, uint32_t i, uint32_t j)
{
    uint32_t m = 0;
    for (uint32_t k = 0; k < s->z; k++)
        if (*fat_at(s, i, j, k) > m)
            m = *fat_at(s, i, j, k);
    return m;
}

/* ------------------------------------------------------- sequential SF_F */

/*
 * Insertion (Section 3.4, used unchanged by SF_F): increment the d Fat
 * counters B_i[h_i][f_i]; B_e^min is the smallest of them after the
 * increment; then every Slim counter A_l[h_l] that equals the minimum of the
 * d Slim counters and is below B_e^min is incremented by one (all tied
 * minima).  A saturated Slim counter (65535) is not incremented.
 */
static void seq_insert(oracle_sketch *s, const uint32_t *h, const uint32_t *f)
{
    uint32_t i;
    for (i = 0; i < s->d; i++)
        *fat_at(s, i, h[i], f[i]) += 1u;
    uint32_t bmin = UINT32_MAX;
    for (i = 0; i < s->d; i++)
        if (*fat_at(s, i, h[i], f[i]) < bmin)
            bmin = *fat_at(s, i, h[i], f[i]);
    uint32_t amin = UINT32_MAX;
    for (i = 0; i < s->d; i++)
        if (*slim_at(s, i, h[i]) < amin)
            amin = *slim_at(s, i, h[i]);
    if (amin < bmin && amin < SLIM_MAX) {
        for (i = 0; i < s->d; i++)
            if (*slim_at(s, i, h[i]) == amin)
                *slim_at(s, i, h[i]) = (uint16_t)(amin + 1u);
    }
}

/*
 * Deletion of SF_F (Section 3.5): decrement B_i[h_i][f_i]; for each row, if
 * the largest counter of bucket B_i[h_i] changed because of it, and A_i[h_i]
 * exceeds the new largest counter, set A_i[h_i] to that value.
 * In checked mode a delete that would take a Fat counter below zero (a
 * strict-turnstile violation) is rejected before anything changes.
 */
static int seq_delete(oracle_sketch *s, const uint32_t *h, const uint32_t *f, int checked)
{
    uint32_t i;
    if (checked)
        for (i = 0; i < s->d; i++)
            if (*fat_at(s, i, h[i], f[i]) == 0)
                return ORACLE_EUNDERFLOW;
    for (i = 0; i < s->d; i++) {
        uint32_t before = bucket_max(s, i, h[i]);
        *fat_at(s, i, h[i], f[i]) -= 1u;
        uint32_t after = bucket_max(s, i, h[i]);
        if (after != before && *slim_at(s, i, h[i]) > after)
            *slim_at(s, i, h[i]) = (uint16_t)after;
    }
    return ORACLE_OK;
}

/* Query (Sections 3.1 and 3.5): the smallest of the d hashed Slim counters. */
static uint32_t query_one(const oracle_sketch *s, const uint32_t *h)
{
    uint32_t q = UINT32_MAX;
    for (uint32_t i = 0; i < s->d; i++)
        if (*slim_at(s, i, h[i]) < q)
            q = *slim_at(s, i, h[i]);
    return q;
}

/* Sequential run over n ops with given indices ([n][d]); ops NULL = inserts. */
int oracle_seq_idx(oracle_sketch *s, const uint32_t *h, const uint32_t *f, const uint8_t *ops,
                   uint64_t n, int checked)
{
    for (uint64_t t = 0; t < n; t++) {
        if (ops && ops[t]) {
            int rc = seq_delete(s, h + t * s->d, f + t * s->d, checked);
            if (rc)
                return rc;
        } else {
            seq_insert(s, h + t * s->d, f + t * s->d);
        }
    }
    return ORACLE_OK;
}

/* Sequential run over n keys (key_bytes each, packed). */
int oracle_seq(oracle_sketch *s, const uint8_t *keys, const uint8_t *ops, uint64_t n, int checked)
{
    uint32_t h[64], f[64];
    if (s->d > 64)
        return ORACLE_EINVAL;
    for (uint64_t t = 0; t < n; t++) {
        key_indices(s, keys + t * s->key_bytes, h, f);
        if (ops && ops[t]) {
            int rc = seq_delete(s, h, f, checked);
            if (rc)
                return rc;
        } else {
            seq_insert(s, h, f);
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------- deterministic batches */

/*
 * batch(b): the op stream is cut into consecutive batches of at most b ops
 * (cut points depend only on op positions; every call starts a new batch).
 * Each batch runs five steps, each over the batch's ops in stream order:
 *
 *  S1 snapshot  for each insert: m0 = min_i A_i[h_i], Bpre_i = B_i[h_i][f_i]
 *               (state before the batch)
 *  S2 Fat +     for each insert: B_i[h_i][f_i] += 1
 *  S3 raise     for each insert: Bmin = min_i B_i[h_i][f_i],
 *               delta = min_i (B_i[h_i][f_i] - Bpre_i),
 *               T = min(m0 + delta, max(m0, Bmin), 65535),
 *               A_i[h_i] = max(A_i[h_i], T) for every row i
 *  S4 Fat -     for each delete: B_i[h_i][f_i] -= 1
 *  S5 clamp     for each delete: A_i[h_i] = min(A_i[h_i], max_k B_i[h_i][k])
 *
 * S3 is the water-level form of the sequential insertion rule: c inserts of
 * one key raise its minimum Slim counters one step at a time while they stay
 * below B_e^min, i.e. to min(m0 + c, max(m0, Bmin)); with one op per batch
 * it is exactly the sequential rule.  S5 is the sequential deletion rule
 * once Appendix I (every A_i[j] <= max_k B_i[j][k]) is taken into account.
 * Every insert (delete) op of the same key computes the same value, so
 * applying S3 (S5) once per op equals applying it once per distinct key.
 */
int oracle_batch_idx(oracle_sketch *s, const uint32_t *h, const uint32_t *f, const uint8_t *ops,
                     uint64_t n, uint64_t b, int checked)
{
    const uint32_t d = s->d;
    if (b == 0)
        return ORACLE_EINVAL;
    uint64_t cap = b < n ? b : n;
    uint32_t *m0 = (uint32_t *)malloc((cap ? cap : 1) * sizeof(uint32_t));
    uint32_t *bpre = (uint32_t *)malloc((cap ? cap : 1) * d * sizeof(uint32_t));
    if (!m0 || !bpre) {
        free(m0);
        free(bpre);
        return ORACLE_ENOMEM;
    }
    int rc = ORACLE_OK;
    for (uint64_t lo = 0; lo < n && rc == ORACLE_OK; lo += b) {
        uint64_t hi = lo + b < n ? lo + b : n;
        uint64_t t;
        uint32_t i;
        /* S1 */
        for (t = lo; t < hi; t++) {
            if (ops && ops[t])
                continue;
            const uint32_t *ht = h + t * d, *ft = f + t * d;
            uint32_t m = UINT32_MAX;
            for (i = 0; i < d; i++) {
                if (*slim_at(s, i, ht[i]) < m)
                    m = *slim_at(s, i, ht[i]);
                bpre[(t - lo) * d + i] = *fat_at(s, i, ht[i], ft[i]);
            }
            m0[t - lo] = m;
        }
        /* S2 */
        for (t = lo; t < hi; t++) {
            if (ops && ops[t])
                continue;
            for (i = 0; i < d; i++)
                *fat_at(s, i, h[t * d + i], f[t * d + i]) += 1u;
        }
        /* S3 */
        for (t = lo; t < hi; t++) {
            if (ops && ops[t])
                continue;
            const uint32_t *ht = h + t * d, *ft = f + t * d;
            uint32_t bmin = UINT32_MAX, delta = UINT32_MAX;
            for (i = 0; i < d; i++) {
                uint32_t post = *fat_at(s, i, ht[i], ft[i]);
                uint32_t grew = post - bpre[(t - lo) * d + i];
                if (post < bmin)
                    bmin = post;
                if (grew < delta)
                    delta = grew;
            }
            uint64_t rise = (uint64_t)m0[t - lo] + delta;
            uint64_t level = m0[t - lo] > bmin ? m0[t - lo] : bmin;
            uint64_t T = rise < level ? rise : level;
            if (T > SLIM_MAX)
                T = SLIM_MAX;
            for (i = 0; i < d; i++)
                if (*slim_at(s, i, ht[i]) < T)
                    *slim_at(s, i, ht[i]) = (uint16_t)T;
        }
        /* S4 */
        for (t = lo; t < hi && rc == ORACLE_OK; t++) {
            if (!(ops && ops[t]))
                continue;
            if (checked)
                for (i = 0; i < d; i++)
                    if (*fat_at(s, i, h[t * d + i], f[t * d + i]) == 0)
                        rc = ORACLE_EUNDERFLOW;
            if (rc)
                break;
            for (i = 0; i < d; i++)
                *fat_at(s, i, h[t * d + i], f[t * d + i]) -= 1u;
        }
        if (rc)
            break;
        /* S5 */
        for (t = lo; t < hi; t++) {
            if (!(ops && ops[t]))
                continue;
            for (i = 0; i < d; i++) {
                uint32_t m = bucket_max(s, i, h[t * d + i]);
                if (*slim_at(s, i, h[t * d + i]) > m)
                    *slim_at(s, i, h[t * d + i]) = (uint16_t)m;
            }
        }
    }
    free(m0);
    free(bpre);
    return rc;
}

/* batch(b) over keys: hashes each batch's keys once, then runs the steps. */
int oracle_batch(oracle_sketch *s, const uint8_t *keys, const uint8_t *ops, uint64_t n, uint64_t b,
                 int checked)
{
    if (b == 0)
        return ORACLE_EINVAL;
    uint64_t cap = b < n ? b : n;
    uint32_t *h = (uint32_t *)malloc((cap ? cap : 1) * s->d * sizeof(uint32_t));
    uint32_t *f = (uint32_t *)malloc((cap ? cap : 1) * s->d * sizeof(uint32_t));
    if (!h || !f) {
        free(h);
        free(f);
        return ORACLE_ENOMEM;
    }
    int rc = ORACLE_OK;
    for (uint64_t lo = 0; lo < n && rc == ORACLE_OK; lo += b) {
        uint64_t m = lo + b < n ? b : n - lo;
        oracle_indices(s, keys + lo * s->key_bytes, m, h, f);
        rc = oracle_batch_idx(s, h, f, ops ? ops + lo : NULL, m, m, checked);
    }
    free(h);
    free(f);
    return rc;
}

/* ------------------------------------------------------------- queries */

void oracle_query_idx(const oracle_sketch *s, const uint32_t *h, uint64_t n, uint32_t *out)
{
    for (uint64_t t = 0; t < n; t++)
        out[t] = query_one(s, h + t * s->d);
}

void oracle_query(const oracle_sketch *s, const uint8_t *keys, uint64_t n, uint32_t *out)
{
    uint32_t h[64], f[64];
    for (uint64_t t = 0; t < n; t++) {
        key_indices(s, keys + t * s->key_bytes, h, f);
        out[t] = query_one(s, h);
    }
}

/* Fat as the plain histogram of the stream: B_i[c_i(e)] += +1 / -1 per op.
 * Used to check the Fat at sizes where running the full sketch is slow. */
void oracle_fat_histogram(const oracle_sketch *s, const uint8_t *keys, const uint8_t *ops,
                          uint64_t n, uint32_t *fat)
{
    uint32_t h[64], f[64];
    for (uint64_t t = 0; t < n; t++) {
        key_indices(s, keys + t * s->key_bytes, h, f);
        for (uint32_t i = 0; i < s->d; i++)
            fat[((uint64_t)i * s->w + h[i]) * s->z + f[i]] += (ops && ops[t]) ? 0xFFFFFFFFu : 1u;
    }
}
