/* Counter-based synthetic input streams (seeded, block-addressable).
 *
 * Word i of stream `seed` is SplitMix64's output function applied to the
 * counter key(seed) + (i + 1) * 0x9E3779B97F4A7C15, where key(seed) is the
 * same output function applied to seed (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Because word i depends on i
 * alone, any byte range of a stream can be regenerated independently.
 *
 *  - uniform bytes: byte j = byte (j % 8) (little endian) of word j / 8;
 *  - residues:      residue j takes the 32-bit half (j % 2) of word j / 2 and
 *                   returns the smallest r with u < cdf[r], where cdf holds the
 *                   cumulative frequency vector scaled to 2^32 (cdf[last] =
 *                   2^32), mapped through an alphabet string.
 *
 * This file produces inputs only; it holds nothing of the membership test. */
#include <stdint.h>
#include <stddef.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t wl_stream_key(uint64_t seed) { return mix64(seed + GAMMA); }

static inline uint64_t word_at(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }

/* out[0..n) = uniform bytes first..first+n of stream `seed`. */
void wl_uniform_bytes(uint64_t seed, uint64_t first, uint64_t n, uint8_t *out) {
    const uint64_t key = wl_stream_key(seed);
    #pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < (int64_t)((n + (1u << 20) - 1) >> 20); ++blk) {
        uint64_t lo = (uint64_t)blk << 20, hi = lo + (1u << 20);
        if (hi > n) hi = n;
        for (uint64_t j = lo; j < hi; ) {
            uint64_t g = first + j;
            uint64_t w = word_at(key, g >> 3);
            unsigned b = (unsigned)(g & 7);
            for (; b < 8 && j < hi; ++b, ++j) out[j] = (uint8_t)(w >> (8 * b));
        }
    }
}

/* out[0..n) = residues first..first+n; cdf has `k` entries (cdf[k-1] = 2^32),
 * letters[r] is the byte emitted for residue r. */
void wl_residues(uint64_t seed, uint64_t first, uint64_t n, const uint64_t *cdf, int k,
                 const uint8_t *letters, uint8_t *out) {
    const uint64_t key = wl_stream_key(seed);
    #pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < (int64_t)((n + (1u << 20) - 1) >> 20); ++blk) {
        uint64_t lo = (uint64_t)blk << 20, hi = lo + (1u << 20);
        if (hi > n) hi = n;
        for (uint64_t j = lo; j < hi; ++j) {
            uint64_t g = first + j;
            uint64_t w = word_at(key, g >> 1);
            uint64_t u = (g & 1) ? (w >> 32) : (w & 0xFFFFFFFFULL);
            int r = 0;
            while (r < k - 1 && u >= cdf[r]) ++r;
            out[j] = letters[r];
        }
    }
}
