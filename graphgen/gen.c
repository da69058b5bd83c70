/*
 * Seeded synthetic graph and workload generators.
 *
 * These produce raw edge lists only (pairs of node ids, possibly with
 * duplicates and self-loops for R-MAT).  They hold none of the estimator
 * arithmetic: cleaning an edge list into a simple connected CSR graph and
 * everything after it belongs to the two implementations that consume
 * these inputs.  The random stream is xoshiro256** seeded through
 * splitmix64 (Blackman and Vigna), independent of the Philox stream the
 * estimators draw from.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { uint64_t s[4]; } gg_rng;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static void rng_seed(gg_rng *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static inline uint64_t rng_next(gg_rng *r) {
    uint64_t *s = r->s;
    uint64_t out = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return out;
}
/* uniform double in [0,1) with 53 random bits */
static inline double rng_unif(gg_rng *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
/* uniform integer in [0,k) by the high half of a 64x64 product */
static inline uint64_t rng_below(gg_rng *r, uint64_t k) {
    return (uint64_t)(((unsigned __int128)rng_next(r) * k) >> 64);
}

/* Erdos-Renyi G(n,p) over unordered pairs i<j, by geometric skipping
 * (Batagelj and Brandes 2005).  Writes at most cap edges; returns the
 * number of edges the stream produced (call again with a larger buffer if
 * it exceeds cap; the output is a deterministic function of the seed). */
int64_t gg_erdos_renyi(int64_t n, double p, uint64_t seed, int64_t cap,
                       int32_t *src, int32_t *dst) {
    gg_rng r; rng_seed(&r, seed);
    if (n < 2 || p <= 0.0) return 0;
    int64_t cnt = 0;
    if (p >= 1.0) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                if (cnt < cap) { src[cnt] = (int32_t)i; dst[cnt] = (int32_t)j; }
                ++cnt;
            }
        return cnt;
    }
    double lq = log1p(-p);
    /* pairs (w, v) with w < v, visited row by row: v = 1..n-1, w = 0..v-1 */
    int64_t v = 1, w = -1;
    while (v < n) {
        double u = rng_unif(&r);
        w += 1 + (int64_t)floor(log1p(-u) / lq);
        while (w >= v && v < n) { w -= v; ++v; }
        if (v < n) {
            if (cnt < cap) { src[cnt] = (int32_t)w; dst[cnt] = (int32_t)v; }
            ++cnt;
        }
    }
    return cnt;
}

/* Barabasi-Albert preferential attachment.  Seed graph: a star with
 * center 0 and leaves 1..m.  Each later node t attaches to m distinct
 * earlier nodes drawn with probability proportional to degree, by
 * sampling uniformly from the list of all edge endpoints so far.
 * Edge count: m + (n-m-1)*m.  Buffers must hold that many edges. */
int64_t gg_barabasi_albert(int64_t n, int64_t m, uint64_t seed,
                           int32_t *src, int32_t *dst) {
    if (m < 1 || n < m + 1) return -1;
    gg_rng r; rng_seed(&r, seed);
    int64_t n_edges = m + (n - m - 1) * m;
    int32_t *ends = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n_edges);
    int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    if (!ends || !pick) { free(ends); free(pick); return -2; }
    int64_t ne = 0, nends = 0;
    for (int64_t j = 1; j <= m; ++j) {
        src[ne] = 0; dst[ne] = (int32_t)j; ++ne;
        ends[nends++] = 0; ends[nends++] = (int32_t)j;
    }
    for (int64_t t = m + 1; t < n; ++t) {
        int64_t got = 0;
        while (got < m) {
            int32_t c = ends[rng_below(&r, (uint64_t)nends)];
            int dup = 0;
            for (int64_t q = 0; q < got; ++q) if (pick[q] == c) { dup = 1; break; }
            if (!dup) pick[got++] = c;
        }
        for (int64_t q = 0; q < m; ++q) {
            src[ne] = (int32_t)t; dst[ne] = pick[q]; ++ne;
            ends[nends++] = (int32_t)t; ends[nends++] = pick[q];
        }
    }
    free(ends); free(pick);
    return ne;
}

/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004), Graph500-style without noise:
 * n_edges = edge_factor * 2^scale directed pairs, each bit level picks a
 * quadrant with probabilities a, b, c, d = 1-a-b-c.  Output is raw: it
 * contains self-loops and duplicates. */
int64_t gg_rmat(int32_t scale, int64_t edge_factor, double a, double b, double c,
                uint64_t seed, int32_t *src, int32_t *dst) {
    if (scale < 1 || scale > 30) return -1;
    gg_rng r; rng_seed(&r, seed);
    int64_t ne = edge_factor << scale;
    double ab = a + b, abc = a + b + c;
    for (int64_t e = 0; e < ne; ++e) {
        uint32_t i = 0, j = 0;
        for (int32_t lvl = 0; lvl < scale; ++lvl) {
            double u = rng_unif(&r);
            uint32_t bi = 0, bj = 0;
            if (u < a) { }
            else if (u < ab) { bj = 1; }
            else if (u < abc) { bi = 1; }
            else { bi = 1; bj = 1; }
            i = (i << 1) | bi; j = (j << 1) | bj;
        }
        src[e] = (int32_t)i; dst[e] = (int32_t)j;
    }
    return ne;
}

/* Connectivity of an undirected edge list over n nodes (union-find), used
 * by the "resample until connected" recipe.  Returns 1 if connected. */
int32_t gg_is_connected(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst) {
    if (n <= 1) return 1;
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!par) return -1;
    for (int64_t i = 0; i < n; ++i) par[i] = (int32_t)i;
    int64_t comps = n;
    for (int64_t e = 0; e < n_edges; ++e) {
        int32_t x = src[e], y = dst[e];
        while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
        while (par[y] != y) { par[y] = par[par[y]]; y = par[y]; }
        if (x != y) { par[x] = y; --comps; }
    }
    free(par);
    return comps == 1 ? 1 : 0;
}
