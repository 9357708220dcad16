/*
 * datagen.c -- seeded, counter-based synthetic column generators.
 *
 * These generators produce the uncompressed input columns that both the CPU
 * oracle and the GPU library consume.  They hold none of the query method's
 * arithmetic: no encoding, no filtering, no joining, no aggregation.
 *
 * Every value is a pure function of (stream, row index), so any slice of a
 * column can be regenerated on its own and generation parallelises.
 *
 * Random source: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  The mixing function and the
 * golden-gamma increment are the published ones.
 *
 *   stream(seed, name) = mix(seed XOR fnv1a64(name))
 *   x_i                = mix(stream + (i + 1) * GAMMA)
 *   uniform[lo, hi]    = lo + floor(x_i * (hi - lo + 1) / 2^64)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t dg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t dg_at(uint64_t stream, uint64_t i) {
    return dg_mix(stream + (i + 1) * DG_GAMMA);
}

/* Map a 64-bit random word onto [lo, hi] (inclusive) by the multiply-shift
 * method; range 0 means the full 2^64 span. */
static inline int64_t dg_scale(uint64_t x, int64_t lo, int64_t hi) {
    uint64_t range = (uint64_t)hi - (uint64_t)lo + 1u;
    if (range == 0) return (int64_t)x;
    uint64_t off = (uint64_t)(((unsigned __int128)x * range) >> 64);
    return (int64_t)((uint64_t)lo + off);
}

uint64_t dg_fnv1a(const char* s) {
    uint64_t h = 0xcbf29ce484222325ULL;
    for (; *s; ++s) {
        h ^= (uint8_t)*s;
        h *= 0x100000001b3ULL;
    }
    return h;
}

uint64_t dg_stream(uint64_t seed, const char* name) {
    return dg_mix(seed ^ dg_fnv1a(name));
}

void dg_raw(uint64_t stream, int64_t row0, int64_t n, uint64_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = dg_at(stream, (uint64_t)(row0 + i));
}

void dg_uniform_i64(uint64_t stream, int64_t row0, int64_t n, int64_t lo, int64_t hi,
                    int64_t* out) {
    for (int64_t i = 0; i < n; ++i)
        out[i] = dg_scale(dg_at(stream, (uint64_t)(row0 + i)), lo, hi);
}

void dg_uniform_i32(uint64_t stream, int64_t row0, int64_t n, int64_t lo, int64_t hi,
                    int32_t* out) {
    for (int64_t i = 0; i < n; ++i)
        out[i] = (int32_t)dg_scale(dg_at(stream, (uint64_t)(row0 + i)), lo, hi);
}

/* Histogram of the n uniform draws [lo, hi] that dg_uniform_* would emit for
 * rows 0..n-1.  counts has hi - lo + 1 entries. */
void dg_hist(uint64_t stream, int64_t n, int64_t lo, int64_t hi, int64_t* counts) {
    int64_t nb = hi - lo + 1;
    memset(counts, 0, (size_t)nb * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        counts[dg_scale(dg_at(stream, (uint64_t)i), lo, hi) - lo] += 1;
}

/* Rows row0..row0+n-1 of the sorted order of the draws summarised by counts:
 * value(i) = lo + smallest d with counts[0] + ... + counts[d] > i. */
void dg_sorted_from_hist(const int64_t* counts, int64_t nbins, int64_t lo, int64_t row0,
                         int64_t n, int64_t* out) {
    int64_t d = 0, cum = counts[0];
    while (d + 1 < nbins && cum <= row0) { ++d; cum += counts[d]; }
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = row0 + i;
        while (d + 1 < nbins && cum <= r) { ++d; cum += counts[d]; }
        out[i] = lo + d;
    }
}

/* Vocabulary of nwords distinct lowercase words, lengths uniform in
 * [minlen, maxlen].  Word k is stored at bytes + k * maxlen, length lens[k].
 * A candidate equal to an earlier word is redrawn from the next counter.
 * Returns 0, or -1 if the word space is too small. */
int dg_vocab(uint64_t seed, int32_t nwords, int32_t minlen, int32_t maxlen, uint8_t* bytes,
             int32_t* lens) {
    uint64_t st = dg_stream(seed, "vocabulary");
    uint64_t ctr = 0;
    for (int32_t k = 0; k < nwords; ++k) {
        for (int attempt = 0;; ++attempt) {
            if (attempt > 1000) return -1;
            uint64_t r = dg_at(st, ctr++);
            int32_t len = (int32_t)dg_scale(dg_at(r, 0), minlen, maxlen);
            uint8_t* w = bytes + (size_t)k * (size_t)maxlen;
            for (int32_t c = 0; c < len; ++c) w[c] = (uint8_t)('a' + dg_scale(dg_at(r, (uint64_t)c + 1), 0, 25));
            int dup = 0;
            for (int32_t j = 0; j < k && !dup; ++j)
                if (lens[j] == len && memcmp(bytes + (size_t)j * (size_t)maxlen, w, (size_t)len) == 0) dup = 1;
            if (!dup) { lens[k] = len; break; }
        }
    }
    return 0;
}

/* Per-row comment draws.  Row i owns the sub-stream r_i = x_i; its draws are
 * mix(r_i + (j + 1) * GAMMA): j = 0 length, j = 1 planting, j >= 2 words. */
static inline int64_t dg_comment_len(uint64_t stream, int64_t row, int32_t minlen, int32_t maxlen) {
    uint64_t r = dg_at(stream, (uint64_t)row);
    return dg_scale(dg_at(r, 0), minlen, maxlen);
}

/* Offsets (n + 1 entries, offsets[0] = 0) of the comment strings of rows
 * row0..row0+n-1; each string has exactly its drawn length. */
void dg_comment_offsets(uint64_t stream, int64_t row0, int64_t n, int32_t minlen, int32_t maxlen,
                        int64_t* offsets) {
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i)
        offsets[i + 1] = offsets[i] + dg_comment_len(stream, row0 + i, minlen, maxlen);
}

/* Comment bytes for rows row0..row0+n-1 at the given offsets: words drawn
 * uniformly from the vocabulary joined by single spaces until the drawn
 * length is reached, then truncated to it.  With probability plant_pct/100
 * a row starts with the plant bytes instead. */
void dg_comment_bytes(uint64_t stream, const uint8_t* vocab, const int32_t* vlens, int32_t nwords,
                      int32_t maxwlen, int64_t row0, int64_t n, int32_t minlen, int32_t maxlen,
                      const uint8_t* plant, int32_t plantlen, int32_t plant_pct,
                      const int64_t* offsets, uint8_t* out) {
    for (int64_t i = 0; i < n; ++i) {
        int64_t row = row0 + i;
        uint64_t r = dg_at(stream, (uint64_t)row);
        int64_t L = dg_scale(dg_at(r, 0), minlen, maxlen);
        uint8_t* dst = out + (offsets[i] - offsets[0]);
        int64_t pos = 0;
        if (plantlen > 0 && dg_scale(dg_at(r, 1), 0, 99) < plant_pct) {
            for (int32_t c = 0; c < plantlen && pos < L; ++c) dst[pos++] = plant[c];
        }
        uint64_t j = 2;
        while (pos < L) {
            if (pos > 0 && dst[pos - 1] != ' ') { dst[pos++] = ' '; if (pos >= L) break; }
            int64_t k = dg_scale(dg_at(r, j++), 0, nwords - 1);
            const uint8_t* w = vocab + (size_t)k * (size_t)maxwlen;
            for (int32_t c = 0; c < vlens[k] && pos < L; ++c) dst[pos++] = w[c];
        }
    }
}
