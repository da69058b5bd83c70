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

/* ------------------------------------------------------------ hyperbolic */
/*
 * Random hyperbolic graph, threshold model (Krioukov, Papadopoulos, Kitsak,
 * Vahdat, Boguna, Phys. Rev. E 82, 2010): n points in a hyperbolic disk of
 * radius R, angles uniform, radii with density alpha sinh(alpha r) /
 * (cosh(alpha R) - 1), alpha = (gamma - 1) / 2; two points are joined when
 * their hyperbolic distance is at most R.  R is set from the target average
 * degree k by the model's large-n relation k = (2/pi) xi^2 n e^{-R/2},
 * xi = alpha / (alpha - 1/2) (requires gamma > 2).
 * Pairs are found band by band (radial bands holding equal numbers of
 * points, each sorted by angle): a point only looks, in each band, at the
 * angular window within which a point of that band's smallest radius could
 * be close enough, then tests the exact distance.  Each edge is emitted once,
 * from its endpoint of smaller (radius, id).
 * Returns the number of edges (written only while below cap), -1 on bad
 * arguments or allocation failure.
 */
typedef struct { double th; double r; int32_t id; } gg_pt;

static int gg_cmp_th(const void *a, const void *b) {
    double x = ((const gg_pt *)a)->th, y = ((const gg_pt *)b)->th;
    return (x > y) - (x < y);
}
static int gg_cmp_r(const void *a, const void *b) {
    double x = ((const gg_pt *)a)->r, y = ((const gg_pt *)b)->r;
    if (x != y) return (x > y) - (x < y);
    return ((const gg_pt *)a)->id - ((const gg_pt *)b)->id;
}

/* largest angular gap at which radii r1, r2 are within distance R */
static double gg_dtheta(double r1, double r2, double coshR) {
    double den = sinh(r1) * sinh(r2);
    if (den <= 0.0) return M_PI;
    double c = (cosh(r1) * cosh(r2) - coshR) / den;
    if (c <= -1.0) return M_PI;
    if (c >= 1.0) return 0.0;
    return acos(c);
}

int64_t gg_hyperbolic(int64_t n, double avg_deg, double gamma, uint64_t seed, int64_t cap,
                      int32_t *src, int32_t *dst) {
    if (n < 2 || avg_deg <= 0.0 || gamma <= 2.0) return -1;
    const double alpha = 0.5 * (gamma - 1.0);
    const double xi = alpha / (alpha - 0.5);
    const double R = 2.0 * log(2.0 * xi * xi * (double)n / (M_PI * avg_deg));
    const double coshR = cosh(R);
    gg_rng rng;
    rng_seed(&rng, seed);
    gg_pt *p = (gg_pt *)malloc(sizeof(gg_pt) * (size_t)n);
    if (!p) return -1;
    const double top = cosh(alpha * R) - 1.0;
    for (int64_t i = 0; i < n; ++i) {
        p[i].th = 2.0 * M_PI * rng_unif(&rng);
        p[i].r = acosh(1.0 + rng_unif(&rng) * top) / alpha;
        p[i].id = (int32_t)i;
    }
    /* bands of equal size in radial order, each sorted by angle */
    qsort(p, (size_t)n, sizeof(gg_pt), gg_cmp_r);
    int64_t nb = 1;
    while ((1LL << nb) < n) ++nb;
    if (nb < 4) nb = 4;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
    double *rmin = (double *)malloc(sizeof(double) * (size_t)nb);
    if (!start || !rmin) { free(p); free(start); free(rmin); return -1; }
    for (int64_t b = 0; b <= nb; ++b) start[b] = b * n / nb;
    for (int64_t b = 0; b < nb; ++b) {
        rmin[b] = start[b] < start[b + 1] ? p[start[b]].r : R;
        qsort(p + start[b], (size_t)(start[b + 1] - start[b]), sizeof(gg_pt), gg_cmp_th);
    }
    int64_t cnt = 0;
    for (int64_t b0 = 0; b0 < nb; ++b0)
        for (int64_t i = start[b0]; i < start[b0 + 1]; ++i) {
            const gg_pt u = p[i];
            const double chu = cosh(u.r), shu = sinh(u.r);
            for (int64_t b = b0; b < nb; ++b) {
                const int64_t lo = start[b], hi = start[b + 1];
                if (lo >= hi) continue;
                const double dth = gg_dtheta(u.r, rmin[b] > u.r ? rmin[b] : u.r, coshR);
                if (dth <= 0.0) continue;
                /* scan the angular window [th - dth, th + dth] (wrapping) */
                double a0 = u.th - dth, a1 = u.th + dth;
                for (int pass = 0; pass < 3; ++pass) {
                    double wl, wh;
                    if (pass == 0) { wl = a0 < 0.0 ? 0.0 : a0; wh = a1 > 2.0 * M_PI ? 2.0 * M_PI : a1; }
                    else if (pass == 1) { if (a0 >= 0.0) continue; wl = a0 + 2.0 * M_PI; wh = 2.0 * M_PI; }
                    else { if (a1 <= 2.0 * M_PI) continue; wl = 0.0; wh = a1 - 2.0 * M_PI; }
                    if (dth >= M_PI) { if (pass > 0) continue; wl = 0.0; wh = 2.0 * M_PI; }
                    int64_t l = lo, h = hi;              /* first index with th >= wl */
                    while (l < h) { int64_t m = (l + h) / 2; if (p[m].th < wl) l = m + 1; else h = m; }
                    for (int64_t j = l; j < hi && p[j].th <= wh; ++j) {
                        const gg_pt w = p[j];
                        if (w.r < u.r || (w.r == u.r && w.id <= u.id)) continue;
                        const double cd = chu * cosh(w.r) - shu * sinh(w.r) * cos(u.th - w.th);
                        if (cd <= coshR) {
                            if (cnt < cap) { src[cnt] = u.id; dst[cnt] = w.id; }
                            ++cnt;
                        }
                    }
                }
            }
        }
    free(p); free(start); free(rmin);
    return cnt;
}

/* The points gg_hyperbolic places for the same arguments (node i's angle and
 * radius), and the disk radius R; for tests that check the pairs by brute force. */
double gg_hyperbolic_points(int64_t n, double avg_deg, double gamma, uint64_t seed, double *th, double *r) {
    if (n < 2 || avg_deg <= 0.0 || gamma <= 2.0) return -1.0;
    const double alpha = 0.5 * (gamma - 1.0);
    const double xi = alpha / (alpha - 0.5);
    const double R = 2.0 * log(2.0 * xi * xi * (double)n / (M_PI * avg_deg));
    gg_rng rng;
    rng_seed(&rng, seed);
    const double top = cosh(alpha * R) - 1.0;
    for (int64_t i = 0; i < n; ++i) {
        th[i] = 2.0 * M_PI * rng_unif(&rng);
        r[i] = acosh(1.0 + rng_unif(&rng) * top) / alpha;
    }
    return R;
}
