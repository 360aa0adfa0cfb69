/*
 * Sequential part of the synthetic stream recipe (input generation only; this
 * file holds none of the sketch's arithmetic).
 *
 * Walk the op positions in order.  A position flagged as a delete candidate
 * removes one live occurrence chosen uniformly (the caller supplies the
 * uniform doubles, one per candidate, so the draw stays numpy-seeded); a
 * candidate with no live occurrence, and every other position, inserts the
 * key pre-drawn for it.  The pool of live occurrences uses swap-remove.
 * This keeps the stream strict-turnstile: no key is deleted more often than
 * it was inserted before that point.
 */
#include <stdint.h>
#include <string.h>

int64_t sfgen_turnstile(const uint8_t *ins_keys, uint64_t n, uint32_t kb,
                        const uint8_t *cand, const double *u_cand,
                        uint8_t *keys_out, uint8_t *ops_out, uint8_t *pool)
{
    uint64_t live = 0, c = 0;
    int64_t ndel = 0;
    for (uint64_t t = 0; t < n; t++) {
        if (cand[t]) {
            double u = u_cand[c++];
            if (live > 0) {
                uint64_t k = (uint64_t)(u * (double)live);
                if (k >= live)
                    k = live - 1;
                memcpy(keys_out + t * kb, pool + k * kb, kb);
                memcpy(pool + k * kb, pool + (live - 1) * kb, kb);
                live--;
                ops_out[t] = 1;
                ndel++;
                continue;
            }
        }
        memcpy(keys_out + t * kb, ins_keys + t * kb, kb);
        memcpy(pool + live * kb, ins_keys + t * kb, kb);
        live++;
        ops_out[t] = 0;
    }
    return ndel;
}
