/*
 * Native draws for the synthetic LP inputs (lpgen.py): the same SplitMix64
 * streams and the same rejection rule, written out in C so that the serving
 * trace (about 9.3e9 entries for 10,000 LPs) can be generated as fast as it is
 * served. Only numbers are drawn here; nothing of the simplex method.
 *
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state advances by the
 * golden-ratio increment and each output is the 64-bit finaliser of the
 * state, so output t (t = 1, 2, ...) of a stream that starts at s0 is
 * mix64(s0 + t * GOLDEN).
 */
#include <stdint.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The start state of LP number k of a run seeded with `seed`. */
uint64_t lpgen_lp_state(uint64_t seed, uint64_t k) { return mix64((seed * GOLDEN) ^ k); }

/*
 * Fills out[0, count) with integers uniform on [lo, hi] (as doubles), taking
 * outputs first+1, first+2, ... of the stream that starts at `state`. With
 * span = hi - lo + 1, an output u is rejected when u >= floor(2^64 / span) *
 * span, else the value is lo + u mod span. Returns the number of outputs
 * consumed (count plus the rejected ones). Needs 1 <= span <= 2^62.
 */
int64_t lpgen_values(uint64_t state, int64_t first, int64_t count, int64_t lo, int64_t hi, double *out) {
    const uint64_t span = (uint64_t)(hi - lo) + 1u;
    /* floor(2^64 / span) * span, or "no rejection" when span divides 2^64 */
    const uint64_t q = UINT64_MAX / span, r = UINT64_MAX % span;
    const int whole = r == span - 1u;
    const uint64_t limit = q * span;
    uint64_t t = (uint64_t)first;
    int64_t i = 0;
    if (span == 1000u) { /* the workloads' range: a constant divisor the compiler turns into a multiply */
        while (i < count) {
            ++t;
            const uint64_t u = mix64(state + t * GOLDEN);
            if (u >= limit) continue;
            out[i++] = (double)(lo + (int64_t)(u % 1000u));
        }
        return (int64_t)(t - (uint64_t)first);
    }
    while (i < count) {
        ++t;
        const uint64_t u = mix64(state + t * GOLDEN);
        if (!whole && u >= limit) continue;
        out[i++] = (double)(lo + (int64_t)(u % span));
    }
    return (int64_t)(t - (uint64_t)first);
}
