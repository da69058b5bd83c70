/*
 * Host-only harness for the oracle's C sampler (oracle/sampler.c), built with
 * AddressSanitizer and UBSan by tests/test_host_sanitizers.py.  It calls every
 * entry point on a few small graphs, with one thread and with several, and
 * checks what must hold whatever the random draws:
 *   - a Wilson sample's next[] is a tree rooted at v, every other node draws
 *     at least once, the per-sample total equals the sum of the draws, and the
 *     block counts add up to the per-sample totals;
 *   - an absorbed walk's visits add up to its length;
 *   - the SpanTree sums, loop-included paths, node-pair and row counts are
 *     the same for every thread count (each sample is computed alone).
 * Prints "ok" and exits 0 when every check passes.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int32_t oracle_wilson(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed, uint32_t stream,
                      uint64_t qid, int64_t sample_begin, int64_t n_samples, int64_t omega_total, int32_t B,
                      int64_t *Y1, int64_t *y1_per_sample, const int64_t *keep_idx, int64_t n_keep,
                      int32_t *next_out, int32_t *draws_out, int32_t n_threads);
int64_t oracle_wilson_ordered(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed,
                              uint32_t stream, uint64_t qid, int64_t sample, const int32_t *order, int64_t n_order,
                              int32_t *next_out, int32_t *draws_out, int32_t *trace, int64_t trace_cap,
                              int64_t *trace_len);
int64_t oracle_loop_included_path(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed,
                                  uint32_t stream, uint64_t qid, int64_t sample, const int32_t *svals,
                                  const int64_t *soff, int32_t s, int32_t *trace, int64_t trace_cap,
                                  int64_t *trace_len);
int32_t oracle_absorbed(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed,
                        uint32_t stream, uint64_t qid, int32_t tag, int64_t walk_begin, int64_t n_walks,
                        int64_t omega_total, int32_t B, int64_t *Y2, int64_t *len_per_walk,
                        int32_t *start_per_walk, int64_t trace_walk, int32_t *trace, int64_t trace_cap,
                        int64_t *trace_len, int32_t n_threads);
int32_t oracle_query_walks(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed,
                           uint32_t stream, uint64_t qid, int32_t start, int32_t sub, int32_t a, int32_t b,
                           int64_t walk_begin, int64_t n_walks, int64_t *dep_a, int64_t *dep_b, double *norm_len,
                           int64_t *len);
int64_t oracle_bfs_tree(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, int32_t *bfs_par);
int32_t oracle_spantree(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed,
                        uint32_t stream, uint64_t qid, int64_t sample_begin, int64_t n_samples, int32_t kind,
                        int64_t *X1, int64_t *X2, int64_t *s1, int64_t *s2, int32_t n_threads);
int32_t oracle_loop_included(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed,
                             uint32_t stream, uint64_t qid, int32_t tag, int64_t sample_begin, int64_t n_paths,
                             int64_t omega_total, int32_t B, int64_t *Y2, int64_t *len_per_path,
                             int32_t n_threads);
int32_t oracle_pair_paths(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed,
                          uint32_t stream, uint64_t qid, int64_t sample_begin, int64_t n_samples,
                          int64_t omega_total, int32_t B, int64_t n_pairs, const int32_t *s, const int32_t *t,
                          int64_t *V, int32_t n_threads);
int32_t oracle_lv_rows(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, uint64_t seed,
                       uint32_t stream, uint64_t qid, int64_t sample_begin, int64_t n_samples, int64_t omega_total,
                       int32_t B, int64_t n_sources, const int32_t *src, int64_t *Y, int32_t n_threads);

static int failures = 0;
#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            fprintf(stderr, "FAIL: " __VA_ARGS__); \
            fprintf(stderr, "\n");                \
            ++failures;                           \
        }                                         \
    } while (0)

typedef struct {
    const char *name;
    int64_t n;
    int64_t *rp;
    int32_t *col;
} graph;

/* CSR from a symmetric 0/1 adjacency matrix (rows ascending, no loops) */
static graph from_adj(const char *name, int64_t n, const uint8_t *adj) {
    graph g = {name, n, (int64_t *)calloc((size_t)n + 1, sizeof(int64_t)), NULL};
    for (int64_t u = 0; u < n; ++u)
        for (int64_t w = 0; w < n; ++w) g.rp[u + 1] += adj[u * n + w];
    for (int64_t u = 0; u < n; ++u) g.rp[u + 1] += g.rp[u];
    g.col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g.rp[n] > 0 ? g.rp[n] : 1));
    int64_t j = 0;
    for (int64_t u = 0; u < n; ++u)
        for (int64_t w = 0; w < n; ++w)
            if (adj[u * n + w]) g.col[j++] = (int32_t)w;
    return g;
}

static void edge(uint8_t *adj, int64_t n, int64_t a, int64_t b) {
    if (a == b) return;
    adj[a * n + b] = 1;
    adj[b * n + a] = 1;
}

static graph path_graph(int64_t n) {
    uint8_t *adj = (uint8_t *)calloc((size_t)(n * n), 1);
    for (int64_t u = 0; u + 1 < n; ++u) edge(adj, n, u, u + 1);
    graph g = from_adj("path", n, adj);
    free(adj);
    return g;
}

static graph grid_graph(int64_t r, int64_t c) {
    const int64_t n = r * c;
    uint8_t *adj = (uint8_t *)calloc((size_t)(n * n), 1);
    for (int64_t i = 0; i < r; ++i)
        for (int64_t j = 0; j < c; ++j) {
            if (i + 1 < r) edge(adj, n, i * c + j, (i + 1) * c + j);
            if (j + 1 < c) edge(adj, n, i * c + j, i * c + j + 1);
        }
    graph g = from_adj("grid", n, adj);
    free(adj);
    return g;
}

/* a path through all nodes (connected) plus random chords */
static graph random_graph(int64_t n, int64_t chords, uint64_t seed) {
    uint8_t *adj = (uint8_t *)calloc((size_t)(n * n), 1);
    for (int64_t u = 0; u + 1 < n; ++u) edge(adj, n, u, u + 1);
    uint64_t x = seed;
    for (int64_t e = 0; e < chords; ++e) {
        x = x * 6364136223846793005ULL + 1442695040888963407ULL;
        const int64_t a = (int64_t)((x >> 33) % (uint64_t)n);
        x = x * 6364136223846793005ULL + 1442695040888963407ULL;
        const int64_t b = (int64_t)((x >> 33) % (uint64_t)n);
        edge(adj, n, a, b);
    }
    graph g = from_adj("random", n, adj);
    free(adj);
    return g;
}

static int same64(const int64_t *a, const int64_t *b, int64_t cnt) {
    return memcmp(a, b, sizeof(int64_t) * (size_t)cnt) == 0;
}

static void check_graph(const graph *g, int32_t root) {
    const int64_t n = g->n, om = 24;
    const int32_t B = 3;
    int64_t keep[3] = {0, 7, om - 1};
    int64_t *Y1[2], *y1[2];
    int32_t *nx = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)n);
    int32_t *dr = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)n);
    const int32_t threads[2] = {1, 3};
    for (int t = 0; t < 2; ++t) {
        Y1[t] = (int64_t *)calloc((size_t)(B * n), sizeof(int64_t));
        y1[t] = (int64_t *)calloc((size_t)om, sizeof(int64_t));
        CHECK(oracle_wilson(n, g->rp, g->col, root, 5, 0, 0, 0, om, om, B, Y1[t], y1[t], keep, 3, nx, dr,
                            threads[t]) == 0,
              "%s: oracle_wilson status", g->name);
    }
    CHECK(same64(Y1[0], Y1[1], B * n) && same64(y1[0], y1[1], om), "%s: wilson differs across threads", g->name);
    int64_t tot = 0, blk = 0;
    for (int64_t i = 0; i < om; ++i) tot += y1[0][i];
    for (int64_t i = 0; i < B * n; ++i) blk += Y1[0][i];
    CHECK(tot == blk, "%s: block counts %lld vs per-sample totals %lld", g->name, (long long)blk, (long long)tot);
    for (int q = 0; q < 3; ++q) {
        const int32_t *nq = nx + q * n, *dq = dr + q * n;
        int64_t sum = 0;
        for (int64_t u = 0; u < n; ++u) {
            sum += dq[u];
            if (u == root) {
                CHECK(nq[u] == -1 && dq[u] == 0, "%s: root entry", g->name);
                continue;
            }
            CHECK(dq[u] >= 1, "%s: node %lld never drew", g->name, (long long)u);
            int64_t x = u, hops = 0;
            while (x != root && hops <= n) {
                x = nq[x];
                ++hops;
                if (x < 0 || x >= n) break;
            }
            CHECK(x == root, "%s: next[] from %lld does not reach the root", g->name, (long long)u);
        }
        CHECK(sum == y1[0][keep[q]], "%s: kept sample draws", g->name);
    }
    /* one sample in a reversed start order gives the same stacks */
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t u = 0; u < n; ++u) order[u] = (int32_t)(n - 1 - u);
    int32_t *no = (int32_t *)malloc(sizeof(int32_t) * (size_t)n), *dn = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t tr[64];
    int64_t tl = 0;
    const int64_t tot7 = oracle_wilson_ordered(n, g->rp, g->col, root, 5, 0, 0, 7, order, n, no, dn, tr, 64, &tl);
    CHECK(tot7 == y1[0][7], "%s: ordered sample total", g->name);
    CHECK(memcmp(no, nx + n, sizeof(int32_t) * (size_t)n) == 0, "%s: ordered sample tree", g->name);
    /* loop-included path from the last node in sample 7 */
    int32_t ptr[4096];
    const int64_t mv = oracle_loop_included_path(n, g->rp, g->col, root, 5, 0, 0, 7, NULL, NULL, (int32_t)(n - 1),
                                                 ptr, 4096, &tl);
    CHECK(mv >= 0, "%s: loop-included path", g->name);

    /* absorbed walks of both kinds */
    for (int tag = 1; tag <= 2; ++tag) {
        int64_t *Y2[2], *len[2];
        for (int t = 0; t < 2; ++t) {
            Y2[t] = (int64_t *)calloc((size_t)(B * n), sizeof(int64_t));
            len[t] = (int64_t *)calloc((size_t)om, sizeof(int64_t));
            int32_t *start = (int32_t *)calloc((size_t)om, sizeof(int32_t));
            int32_t wt[256];
            int64_t wl = 0;
            CHECK(oracle_absorbed(n, g->rp, g->col, root, 5, 0, 0, tag, 0, om, om, B, Y2[t], len[t], start, 3, wt,
                                  256, &wl, threads[t]) == 0,
                  "%s: absorbed status", g->name);
            free(start);
        }
        CHECK(same64(Y2[0], Y2[1], B * n) && same64(len[0], len[1], om), "%s: absorbed differs", g->name);
        int64_t lsum = 0, vsum = 0;
        for (int64_t i = 0; i < om; ++i) lsum += len[0][i];
        for (int64_t i = 0; i < B * n; ++i) vsum += Y2[0][i];
        CHECK(lsum == vsum, "%s: absorbed visits vs lengths", g->name);
        for (int t = 0; t < 2; ++t) {
            free(Y2[t]);
            free(len[t]);
        }
    }
    /* query walks */
    int64_t da[8], db[8], ln[8];
    double nl[8];
    CHECK(oracle_query_walks(n, g->rp, g->col, root, 5, 0, 9, (int32_t)(n - 1), 0, (int32_t)(n - 1), (int32_t)(n / 2),
                             0, 8, da, db, nl, ln) == 0,
          "%s: query walks", g->name);
    /* BFS tree and SpanTree sums */
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    CHECK(oracle_bfs_tree(n, g->rp, g->col, root, par) == n, "%s: BFS reaches every node", g->name);
    for (int kind = 1; kind <= 2; ++kind) {
        int64_t *X1[2], *X2[2], *s1[2], *s2[2];
        for (int t = 0; t < 2; ++t) {
            X1[t] = (int64_t *)calloc((size_t)n, sizeof(int64_t));
            X2[t] = (int64_t *)calloc((size_t)n, sizeof(int64_t));
            s1[t] = (int64_t *)calloc((size_t)om, sizeof(int64_t));
            s2[t] = (int64_t *)calloc((size_t)om, sizeof(int64_t));
            CHECK(oracle_spantree(n, g->rp, g->col, root, 5, 0, 0, 0, om, kind, X1[t], X2[t], s1[t], s2[t],
                                  threads[t]) == 0,
                  "%s: spantree status", g->name);
        }
        CHECK(same64(X1[0], X1[1], n) && same64(X2[0], X2[1], n) && same64(s1[0], s1[1], om) &&
                  same64(s2[0], s2[1], om),
              "%s: spantree differs across threads", g->name);
        for (int t = 0; t < 2; ++t) {
            free(X1[t]);
            free(X2[t]);
            free(s1[t]);
            free(s2[t]);
        }
    }
    /* loop-included paths, node pairs and rows */
    int32_t ps[4] = {0, (int32_t)(n - 1), (int32_t)(n / 2), root}, pt[4] = {(int32_t)(n - 1), 1, (int32_t)(n / 3), 0};
    int64_t *Lp[2], *Ll[2], *V[2], *R[2];
    for (int t = 0; t < 2; ++t) {
        Lp[t] = (int64_t *)calloc((size_t)(B * n), sizeof(int64_t));
        Ll[t] = (int64_t *)calloc((size_t)om, sizeof(int64_t));
        V[t] = (int64_t *)calloc((size_t)(B * 4 * 4), sizeof(int64_t));
        R[t] = (int64_t *)calloc((size_t)(B * 2 * n), sizeof(int64_t));
        CHECK(oracle_loop_included(n, g->rp, g->col, root, 5, 0, 0, 1, 0, om, om, B, Lp[t], Ll[t], threads[t]) == 0,
              "%s: loop-included status", g->name);
        CHECK(oracle_pair_paths(n, g->rp, g->col, root, 5, 0, 0, 0, om, om, B, 4, ps, pt, V[t], threads[t]) == 0,
              "%s: pair paths status", g->name);
        CHECK(oracle_lv_rows(n, g->rp, g->col, root, 5, 0, 0, 0, om, om, B, 2, ps, R[t], threads[t]) == 0,
              "%s: rows status", g->name);
    }
    CHECK(same64(Lp[0], Lp[1], B * n) && same64(Ll[0], Ll[1], om), "%s: loop-included differs", g->name);
    CHECK(same64(V[0], V[1], B * 16), "%s: pair sums differ", g->name);
    CHECK(same64(R[0], R[1], B * 2 * n), "%s: rows differ", g->name);
    for (int t = 0; t < 2; ++t) {
        free(Y1[t]);
        free(y1[t]);
        free(Lp[t]);
        free(Ll[t]);
        free(V[t]);
        free(R[t]);
    }
    free(nx);
    free(dr);
    free(order);
    free(no);
    free(dn);
    free(par);
}

int main(void) {
    graph gs[4] = {path_graph(200), grid_graph(6, 7), random_graph(300, 900, 11), random_graph(2, 0, 1)};
    const int32_t roots[4] = {0, 20, 150, 1};
    for (int i = 0; i < 4; ++i) {
        check_graph(&gs[i], roots[i]);
        free(gs[i].rp);
        free(gs[i].col);
    }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
