/*
 * Seeded synthetic graph generators (R-MAT, Erdos-Renyi G(n,M), Barabasi-Albert).
 *
 * This module only produces edge lists.  It holds none of the triangle
 * counting arithmetic: cleaning (self-loop and duplicate removal,
 * symmetrisation), orientation and counting belong to the consumers.  Both
 * the CPU checker and the device path read the same arrays produced here.
 *
 * Randomness is counter based: draw(key, i) is output i of a SplitMix64
 * generator whose state starts at `key` (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), i.e. the finaliser applied
 * to key + (i + 1) * golden_gamma.  Any edge can therefore be generated
 * independently of the others, which makes the large generators parallel and
 * reproducible for any thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Output i of the SplitMix64 stream that starts at state `key`. */
static inline uint64_t gg_draw(uint64_t key, uint64_t i) {
    return gg_mix(key + (i + 1) * GG_GAMMA);
}

/* Stream key for (seed, family tag, sub-stream); tags keep the families apart. */
uint64_t gg_stream_key(uint64_t seed, uint64_t tag, uint64_t sub) {
    return gg_mix(gg_mix(seed ^ (tag * GG_GAMMA)) + sub * 0xD1B54A32D192ED03ULL);
}

uint64_t gg_splitmix64(uint64_t x) { return gg_mix(x + GG_GAMMA); }

/* Uniform integer in [0, bound) from the top 32 bits of a draw (multiply-shift;
 * the bias is below 2^-32 * bound and irrelevant for these workloads). */
static inline uint32_t gg_below(uint64_t r, uint32_t bound) {
    return (uint32_t)(((r >> 32) * (uint64_t)bound) >> 32);
}

enum { TAG_RMAT = 1, TAG_ER = 2, TAG_BA = 3 };

/*
 * R-MAT: `m` samples on 2^scale vertices.  Each sample descends `scale`
 * levels; at each level one 32-bit uniform u picks quadrant
 *   a: u < A, b: u < A+B, c: u < A+B+C, d: otherwise
 * with the thresholds given as 32-bit fixed point (p * 2^32).  Quadrant b sets
 * the destination bit, c the source bit, d both.  Two levels use one 64-bit
 * draw.  No noise and no id permutation.
 */
int gg_rmat(uint32_t scale, uint64_t m, uint64_t seed,
            uint32_t ta, uint32_t tab, uint32_t tabc,
            uint32_t* src, uint32_t* dst) {
    if (scale == 0 || scale > 32) return 1;
    const uint64_t key = gg_stream_key(seed, TAG_RMAT, scale);
    const uint64_t per = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)m; ++e) {
        uint64_t s = 0, d = 0;
        for (uint32_t lv = 0; lv < scale; ++lv) {
            uint64_t r = gg_draw(key, (uint64_t)e * per + (lv >> 1));
            uint32_t u = (lv & 1) ? (uint32_t)(r >> 32) : (uint32_t)r;
            uint32_t sb, db;
            if (u < ta)        { sb = 0; db = 0; }
            else if (u < tab)  { sb = 0; db = 1; }
            else if (u < tabc) { sb = 1; db = 0; }
            else               { sb = 1; db = 1; }
            s = (s << 1) | sb;
            d = (d << 1) | db;
        }
        src[e] = (uint32_t)s;
        dst[e] = (uint32_t)d;
    }
    return 0;
}

/* Erdos-Renyi G(n, M) by pair sampling: M uniform (u, v) pairs, which may
 * include self-loops and repeats (removed by the consumer's cleaning). */
int gg_er(uint32_t n, uint64_t m, uint64_t seed, uint32_t* src, uint32_t* dst) {
    if (n == 0) return 1;
    const uint64_t key = gg_stream_key(seed, TAG_ER, n);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)m; ++e) {
        src[e] = gg_below(gg_draw(key, 2 * (uint64_t)e), n);
        dst[e] = gg_below(gg_draw(key, 2 * (uint64_t)e + 1), n);
    }
    return 0;
}

/*
 * Barabasi-Albert preferential attachment with the repeated-endpoint list of
 * Batagelj and Brandes ("Efficient generation of large random networks",
 * Phys. Rev. E 71, 2005): picking a uniform entry of the list of all edge
 * endpoints picks a vertex with probability proportional to its degree.
 * Seed graph: the complete graph on vertices 0..k (k = edges per new vertex).
 * Each later vertex v attaches to k distinct earlier vertices.
 * Output: exactly gg_ba_edges(n, k) edges.
 */
uint64_t gg_ba_edges(uint32_t n, uint32_t k) {
    if (n <= k + 1) return (uint64_t)n * (n - (n > 0)) / 2;
    return (uint64_t)(k + 1) * k / 2 + (uint64_t)(n - k - 1) * k;
}

int gg_ba(uint32_t n, uint32_t k, uint64_t seed, uint32_t* src, uint32_t* dst) {
    if (k == 0 || k > 1024) return 1;
    const uint64_t key = gg_stream_key(seed, TAG_BA, ((uint64_t)n << 16) | k);
    const uint64_t total = gg_ba_edges(n, k);
    uint32_t* ends = (uint32_t*)malloc(sizeof(uint32_t) * 2 * (total + 1));
    if (!ends) return 2;
    uint64_t e = 0;
    uint32_t seedn = n < k + 1 ? n : k + 1;
    for (uint32_t a = 0; a < seedn; ++a)
        for (uint32_t b = a + 1; b < seedn; ++b) {
            src[e] = a; dst[e] = b;
            ends[2 * e] = a; ends[2 * e + 1] = b;
            ++e;
        }
    uint32_t picks[1024];
    uint64_t ctr = 0;
    for (uint32_t v = seedn; v < n; ++v) {
        const uint64_t nends = 2 * e;  /* endpoints of edges placed before v */
        uint32_t got = 0;
        while (got < k) {
            uint64_t r = gg_draw(key, ctr++);
            uint32_t t = ends[(uint64_t)(((unsigned __int128)r * nends) >> 64)];
            int dup = 0;
            for (uint32_t j = 0; j < got; ++j) dup |= (picks[j] == t);
            if (!dup) picks[got++] = t;
        }
        for (uint32_t j = 0; j < k; ++j) {
            src[e] = v; dst[e] = picks[j];
            ends[2 * e] = v; ends[2 * e + 1] = picks[j];
            ++e;
        }
    }
    free(ends);
    return 0;
}
