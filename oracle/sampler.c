/*
 * CPU ORACLE -- test infrastructure only.  Only tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code with the HIP library.
 *
 * Plain, scalar, sequential implementation of the sampling side of the
 * loop-erased-walk estimators of "Scalable Algorithms for Laplacian
 * Pseudo-inverse Computation" (arXiv 2311.10290):
 *   - Wilson's algorithm LE_v rooted at the landmark v with the per-node stack
 *     view of its random choices (Sec. 3.4; LEWalk-ECC algorithm, Alg. 2,
 *     sampling phase; LEWalk-KC, Alg. 4, first line of the loop body);
 *   - v-absorbed walks from a uniform start (Alg. 2, second phase) or from a
 *     start drawn from the stationary distribution (Alg. 4);
 *   - loop-included paths read from the stacks (Sec. 3.4, Fig. 1(d)).
 *   - loop-included paths from given node pairs, the counts behind entries of
 *     L_v^{-1} and effective resistances (Sec. 3.4, Sec. 2), and from given
 *     sources, the counts behind whole rows of L_v^{-1}.
 * Random choices (the paper leaves the generator open):
 *   - generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11);
 *   - key = (seed, stream<<32 | root);
 *   - the k-th draw at node u in Wilson sample i is stack entry S[u][k],
 *     counter (i | 0<<56, u, k, qid), so the sampled stacks do not depend on
 *     the order in which walks are run (Wilson's stack argument, Sec. 3.4);
 *   - absorbed walk i of kind tag (1 = uniform start, 2 = stationary start)
 *     uses counter (i | tag<<56, t, 0, qid) for its t-th draw; t = 0 picks the
 *     start;
 *   - a draw x in [0, 2^64) picks index floor(x * d / 2^64) among d choices
 *     (the u's neighbours in ascending order, or the n nodes, or the 2m CSR
 *     slots for a stationary start).
 * Counts are exact 64-bit integers; dividing by degrees and sample sizes is
 * left to the FP64 estimator assembly (oracle/estimators.py).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------ Philox4x64-10 */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                             uint64_t k0, uint64_t k1) {
    uint64_t ctr[4] = {c0, c1, c2, c3}, key[2] = {k0, k1}, out[4];
    oracle_philox4x64_10(ctr, key, out);
    return out[0];
}

/* index in [0, d) for a 64-bit draw x */
uint64_t oracle_map_below(uint64_t x, uint64_t d) {
    return (uint64_t)(((unsigned __int128)x * d) >> 64);
}

/* ------------------------------------------------------------ draw sources */
typedef struct {
    const int64_t *rp; const int32_t *col;
    uint64_t k0, k1;     /* Philox key */
    uint64_t c0;         /* sample index | tag<<56 */
    uint64_t qid;
    /* scripted stacks (tests): S[u] = vals[off[u] .. off[u+1]) */
    const int32_t *svals; const int64_t *soff;
    int failed;
} draw_ctx;

/* k-th entry of the stack S[u] of the current Wilson sample */
static int32_t stack_entry(draw_ctx *c, int32_t u, int64_t k) {
    if (c->svals) {
        if (c->soff[u] + k >= c->soff[u + 1]) { c->failed = 1; return -1; }
        return c->svals[c->soff[u] + k];
    }
    uint64_t x = philox_word0(c->c0, (uint64_t)u, (uint64_t)k, c->qid, c->k0, c->k1);
    int64_t d = c->rp[u + 1] - c->rp[u];
    return c->col[c->rp[u] + (int64_t)oracle_map_below(x, (uint64_t)d)];
}

static uint64_t make_key1(uint32_t stream, int32_t root) {
    return ((uint64_t)stream << 32) | (uint64_t)(uint32_t)root;
}

/* ------------------------------------------------------------ Wilson LE_v */
/* One loop-erased-walk sample rooted at `root` (Alg. 2, sampling phase).
 * Starts are taken in `order` (n_order nodes), default ascending ids
 * skipping the root.  On return draws[u] = number of draws at u (the node's
 * count in y1 before normalisation), next[u] = its tree parent (-1 for the
 * root).  Optionally records the trajectory (each walk's visited nodes and
 * the tree node it stops at).  Returns the total number of draws, or -1 if a
 * scripted stack ran out. */
static int64_t wilson_sample(int64_t n, int32_t root, draw_ctx *dc,
                             const int32_t *order, int64_t n_order,
                             uint8_t *intree, int32_t *next, int32_t *draws,
                             int32_t *trace, int64_t trace_cap, int64_t *trace_len) {
    memset(intree, 0, (size_t)n);
    for (int64_t i = 0; i < n; ++i) { next[i] = -1; draws[i] = 0; }
    intree[root] = 1;
    int64_t total = 0, tl = 0;
    int64_t n_starts = order ? n_order : n;
    for (int64_t j = 0; j < n_starts; ++j) {
        int32_t start = order ? order[j] : (int32_t)j;
        if (!order && start == root) continue;
        int32_t u = start;
        if (intree[u]) continue;
        /* walk until the tree is hit, overwriting next[] (loops erase themselves) */
        while (!intree[u]) {
            int32_t w = stack_entry(dc, u, draws[u]);
            if (dc->failed) return -1;
            draws[u] += 1;
            next[u] = w;
            if (trace) { if (tl < trace_cap) trace[tl] = u; ++tl; }
            ++total;
            u = w;
        }
        if (trace) { if (tl < trace_cap) trace[tl] = u; ++tl; }
        /* retrace from the start along next[]: the loop-erased path joins the tree */
        u = start;
        while (!intree[u]) { intree[u] = 1; u = next[u]; }
    }
    if (trace_len) *trace_len = tl;
    return total;
}

/*
 * omega-sample driver.  Samples [sample_begin, sample_begin + n_samples) of a
 * run of omega_total samples; sample i adds its draw counts into block
 * b = floor(i * B / omega_total) of Y1 ([B][n], may be NULL).  y1_per_sample
 * ([n_samples], may be NULL) receives each sample's total draws.  For the
 * samples listed in keep_idx (absolute indices) the per-node next[] and
 * draws[] arrays are copied to next_out/draws_out ([n_keep][n]).
 * Returns 0, or -1 on allocation failure.
 */
int32_t oracle_wilson(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                      uint64_t seed, uint32_t stream, uint64_t qid,
                      int64_t sample_begin, int64_t n_samples, int64_t omega_total, int32_t B,
                      int64_t *Y1, int64_t *y1_per_sample,
                      const int64_t *keep_idx, int64_t n_keep, int32_t *next_out, int32_t *draws_out,
                      int32_t n_threads) {
    int32_t status = 0;
    if (B < 1) B = 1;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads)
#endif
    {
        uint8_t *intree = (uint8_t *)malloc((size_t)n);
        int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *draws = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int64_t *acc = Y1 ? (int64_t *)calloc((size_t)n, sizeof(int64_t)) : NULL;
        int64_t acc_block = -1;
        if (!intree || !next || !draws || (Y1 && !acc)) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            status = -1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int64_t s = 0; s < n_samples; ++s) {
                int64_t i = sample_begin + s;
                draw_ctx dc;
                memset(&dc, 0, sizeof dc);
                dc.rp = rp; dc.col = col; dc.k0 = seed; dc.k1 = make_key1(stream, root);
                dc.c0 = (uint64_t)i; dc.qid = qid;
                int64_t tot = wilson_sample(n, root, &dc, NULL, 0, intree, next, draws, NULL, 0, NULL);
                if (y1_per_sample) y1_per_sample[s] = tot;
                if (Y1) {
                    int64_t b = (int64_t)(((__int128)i * B) / omega_total);
                    if (b != acc_block) {
                        if (acc_block >= 0) {
#ifdef _OPENMP
#pragma omp critical(oracle_y1)
#endif
                            for (int64_t u = 0; u < n; ++u) { Y1[acc_block * n + u] += acc[u]; acc[u] = 0; }
                        }
                        acc_block = b;
                    }
                    for (int64_t u = 0; u < n; ++u) acc[u] += draws[u];
                }
                for (int64_t q = 0; q < n_keep; ++q)
                    if (keep_idx[q] == i) {
                        memcpy(next_out + q * n, next, sizeof(int32_t) * (size_t)n);
                        memcpy(draws_out + q * n, draws, sizeof(int32_t) * (size_t)n);
                    }
            }
            if (Y1 && acc_block >= 0) {
#ifdef _OPENMP
#pragma omp critical(oracle_y1)
#endif
                for (int64_t u = 0; u < n; ++u) Y1[acc_block * n + u] += acc[u];
            }
        }
        free(intree); free(next); free(draws); free(acc);
    }
    return status;
}

/* One Wilson sample with an explicit start order (order-independence tests). */
int64_t oracle_wilson_ordered(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                              uint64_t seed, uint32_t stream, uint64_t qid, int64_t sample,
                              const int32_t *order, int64_t n_order,
                              int32_t *next_out, int32_t *draws_out,
                              int32_t *trace, int64_t trace_cap, int64_t *trace_len) {
    uint8_t *intree = (uint8_t *)malloc((size_t)n);
    if (!intree) return -2;
    draw_ctx dc;
    memset(&dc, 0, sizeof dc);
    dc.rp = rp; dc.col = col; dc.k0 = seed; dc.k1 = make_key1(stream, root);
    dc.c0 = (uint64_t)sample; dc.qid = qid;
    int64_t tot = wilson_sample(n, root, &dc, order, n_order, intree, next_out, draws_out,
                                trace, trace_cap, trace_len);
    free(intree);
    return tot;
}

/* One Wilson run over explicitly given stacks (worked-example tests). */
int64_t oracle_wilson_scripted(int64_t n, int32_t root, const int32_t *svals, const int64_t *soff,
                               const int32_t *order, int64_t n_order,
                               int32_t *next_out, int32_t *draws_out,
                               int32_t *trace, int64_t trace_cap, int64_t *trace_len) {
    uint8_t *intree = (uint8_t *)malloc((size_t)n);
    if (!intree) return -2;
    draw_ctx dc;
    memset(&dc, 0, sizeof dc);
    dc.svals = svals; dc.soff = soff;
    int64_t tot = wilson_sample(n, root, &dc, order, n_order, intree, next_out, draws_out,
                                trace, trace_cap, trace_len);
    free(intree);
    return tot;
}

/* Loop-included path P[s] of a Wilson sample (Sec. 3.4, Fig. 1(d)): from s,
 * jump to the lowest unread entry of the current node's stack, until the
 * root.  With svals == NULL the stacks are those of Wilson sample `sample`
 * (Philox keyed as above).  Writes the node sequence (s ... root) and returns
 * its number of moves, or -1 if a scripted stack ran out / -2 on failure. */
int64_t oracle_loop_included_path(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                                  uint64_t seed, uint32_t stream, uint64_t qid, int64_t sample,
                                  const int32_t *svals, const int64_t *soff, int32_t s,
                                  int32_t *trace, int64_t trace_cap, int64_t *trace_len) {
    int64_t *pos = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!pos) return -2;
    draw_ctx dc;
    memset(&dc, 0, sizeof dc);
    dc.rp = rp; dc.col = col; dc.k0 = seed; dc.k1 = make_key1(stream, root);
    dc.c0 = (uint64_t)sample; dc.qid = qid; dc.svals = svals; dc.soff = soff;
    int64_t moves = 0, tl = 0;
    int32_t u = s;
    while (u != root) {
        if (tl < trace_cap) trace[tl] = u;
        ++tl;
        int32_t w = stack_entry(&dc, u, pos[u]);
        if (dc.failed) { free(pos); return -1; }
        pos[u] += 1;
        ++moves;
        u = w;
    }
    if (tl < trace_cap) trace[tl] = u;
    ++tl;
    if (trace_len) *trace_len = tl;
    free(pos);
    return moves;
}

/* ------------------------------------------------------------ absorbed walks */
/* The t-th draw of absorbed walk i of kind tag. */
static uint64_t walk_draw(uint64_t k0, uint64_t k1, uint64_t tag, uint64_t i, uint64_t t, uint64_t sub,
                          uint64_t qid) {
    return philox_word0(i | (tag << 56), t, sub, qid, k0, k1);
}

/*
 * v-absorbed walks (Alg. 2 second phase for tag 1; Alg. 4 for tag 2).
 * Walk i in [walk_begin, walk_begin + n_walks): start s = floor(x0 * n / 2^64)
 * (tag 1, uniform over all of V) or s = col[floor(x0 * 2m / 2^64)] (tag 2,
 * probability d_s / 2m), then move to a uniform neighbour until the root is
 * reached.  Every departure from a node u counts one visit of u (the walk's
 * contribution to y2 before normalisation) and one unit of length.
 * Y2 ([B][n], may be NULL) gets the visits in block floor(i*B/omega_total);
 * len_per_walk ([n_walks], may be NULL) the lengths; start_per_walk the
 * starts.  If trace != NULL the node sequence of walk trace_walk is recorded.
 */
int32_t oracle_absorbed(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                        uint64_t seed, uint32_t stream, uint64_t qid, int32_t tag,
                        int64_t walk_begin, int64_t n_walks, int64_t omega_total, int32_t B,
                        int64_t *Y2, int64_t *len_per_walk, int32_t *start_per_walk,
                        int64_t trace_walk, int32_t *trace, int64_t trace_cap, int64_t *trace_len,
                        int32_t n_threads) {
    if (B < 1) B = 1;
    uint64_t k0 = seed, k1 = make_key1(stream, root);
    int64_t nnz = rp[n];
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(n_threads)
#endif
    for (int64_t w = 0; w < n_walks; ++w) {
        int64_t i = walk_begin + w;
        uint64_t x0 = walk_draw(k0, k1, (uint64_t)tag, (uint64_t)i, 0, 0, qid);
        int32_t s;
        if (tag == 1) s = (int32_t)oracle_map_below(x0, (uint64_t)n);
        else if (nnz > 0) s = col[oracle_map_below(x0, (uint64_t)nnz)];
        else s = root;   /* a single node without edges: the walk is empty */
        if (start_per_walk) start_per_walk[w] = s;
        int64_t b = (int64_t)(((__int128)i * B) / omega_total);
        int32_t u = s;
        int64_t len = 0, tl = 0;
        int rec = (trace && i == trace_walk);
        while (u != root) {
            if (rec) { if (tl < trace_cap) trace[tl] = u; ++tl; }
            if (Y2) {
#ifdef _OPENMP
#pragma omp atomic
#endif
                Y2[b * n + u] += 1;
            }
            ++len;
            uint64_t x = walk_draw(k0, k1, (uint64_t)tag, (uint64_t)i, (uint64_t)len, 0, qid);
            int64_t d = rp[u + 1] - rp[u];
            u = col[rp[u] + (int64_t)oracle_map_below(x, (uint64_t)d)];
        }
        if (rec) { if (tl < trace_cap) trace[tl] = u; ++tl; *trace_len = tl; }
        if (len_per_walk) len_per_walk[w] = len;
    }
    return 0;
}

/* ------------------------------------------------------------ query walks */
/*
 * Walks for single-node and pairwise queries (Lemma 1, and the normalised
 * path length lemma of Sec. 4.3).  Walk i (sub-stream sub = 0 from a, 1 from
 * b) starts at its given node and moves to uniform neighbours until the root;
 * its j-th move (j = 1, 2, ...) uses counter (i | 3<<56, j, sub, qid).  For
 * every walk: the number of departures from a and from b, and the sum of
 * 1/d_x over its departures x (accumulated in FP64 in walk order).
 * Outputs [n_walks] each; NULL skips.
 */
int32_t oracle_query_walks(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                           uint64_t seed, uint32_t stream, uint64_t qid, int32_t start, int32_t sub,
                           int32_t a, int32_t b, int64_t walk_begin, int64_t n_walks,
                           int64_t *dep_a, int64_t *dep_b, double *norm_len, int64_t *len) {
    (void)n;
    uint64_t k0 = seed, k1 = make_key1(stream, root);
    for (int64_t w = 0; w < n_walks; ++w) {
        int64_t i = walk_begin + w;
        int32_t u = start;
        int64_t da = 0, db = 0, steps = 0;
        double nl = 0.0;
        while (u != root) {
            int64_t d = rp[u + 1] - rp[u];
            if (u == a) ++da;
            if (u == b) ++db;
            nl += 1.0 / (double)d;
            ++steps;
            uint64_t x = walk_draw(k0, k1, 3, (uint64_t)i, (uint64_t)steps, (uint64_t)sub, qid);
            u = col[rp[u] + (int64_t)oracle_map_below(x, (uint64_t)d)];
        }
        if (dep_a) dep_a[w] = da;
        if (dep_b) dep_b[w] = db;
        if (norm_len) norm_len[w] = nl;
        if (len) len[w] = steps;
    }
    return 0;
}

/* ------------------------------------------------------------ SpanTree (Alg. 1, Alg. 3) */
/* BFS tree from the root, neighbours taken in ascending order: bfs_par[u] is
 * u's parent (-1 at the root).  Returns the number of nodes reached. */
int64_t oracle_bfs_tree(int64_t n, const int64_t *rp, const int32_t *col, int32_t root, int32_t *bfs_par) {
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *seen = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!queue || !seen) { free(queue); free(seen); return -1; }
    for (int64_t i = 0; i < n; ++i) bfs_par[i] = -1;
    int64_t head = 0, tail = 0;
    queue[tail++] = root;
    seen[root] = 1;
    while (head < tail) {
        int32_t a = queue[head++];
        for (int64_t j = rp[a]; j < rp[a + 1]; ++j) {
            int32_t b = col[j];
            if (!seen[b]) { seen[b] = 1; bfs_par[b] = a; queue[tail++] = b; }
        }
    }
    free(queue); free(seen);
    return tail;
}

/*
 * The per-tree part of Alg. 1 (weights w = 1) and Alg. 3 (w = degrees) for
 * one spanning tree next[] rooted at `root` (next[root] = -1):
 *   1. path support: ps[a] = sum of w[u] over the nodes u whose tree path
 *      to the root uses the out-edge (a, next[a]) -- the flow on that edge
 *      when w[u] enters at every u and leaves at the root (in units of 1/sum w);
 *   2. a depth-first traversal of the tree from the root gives visit and
 *      finish times; a is an ancestor-or-self of u iff u's interval lies in a's;
 *   3. for every u, along the BFS path from u to the root, each edge (e1, e2)
 *      that is a tree edge on u's own tree path (its lower end an
 *      ancestor-or-self of u) adds the flow it carries in the direction
 *      e1 -> e2: +1 to x1[u] and +ps[e1] to x2[u] if next[e1] = e2, -1 and
 *      -ps[e2] if next[e2] = e1.
 * x1[u] averages to (L_v^{-1})_uu and x2[u] / sum w to the voltage at u of the
 * weighted system (Sec. 4.1, Sec. 5.2).  Scratch: 5n int32 and n+1 int64
 * (child lists); vis/fin are its first two n-blocks.  x1, x2, ps are
 * written, not accumulated.
 */
void oracle_spantree_tree(int64_t n, const int32_t *next, int32_t root, const int32_t *bfs_par,
                          const int64_t *w, int64_t *ps, int64_t *x1, int64_t *x2,
                          int32_t *scratch, int64_t *kid_off) {
    int32_t *vis = scratch, *fin = scratch + n, *kids = scratch + 2 * n, *stack = scratch + 3 * n,
            *it = scratch + 4 * n;   /* it[a]: next child of a to visit */
    /* 1. path support, walking every node's tree path */
    for (int64_t a = 0; a < n; ++a) ps[a] = 0;
    for (int64_t u = 0; u < n; ++u)
        for (int32_t a = (int32_t)u; a != root; a = next[a]) ps[a] += w[u];
    /* 2. DFS from the root over child lists (children in ascending id) */
    for (int64_t i = 0; i <= n; ++i) kid_off[i] = 0;
    for (int64_t u = 0; u < n; ++u)
        if (u != root) kid_off[next[u] + 1] += 1;
    for (int64_t i = 0; i < n; ++i) kid_off[i + 1] += kid_off[i];
    for (int64_t i = 0; i < n; ++i) stack[i] = 0;           /* fill cursors */
    for (int64_t u = 0; u < n; ++u)
        if (u != root) kids[kid_off[next[u]] + stack[next[u]]++] = (int32_t)u;
    int32_t clock = 0, top = 0;
    /* iterative DFS: stack holds nodes; vis set on entry, fin on exit */
    for (int64_t i = 0; i < n; ++i) { vis[i] = -1; fin[i] = -1; }
    for (int64_t i = 0; i < n; ++i) it[i] = 0;
    stack[top++] = root;
    vis[root] = clock++;
    while (top > 0) {
        int32_t a = stack[top - 1];
        if (kid_off[a] + it[a] < kid_off[a + 1]) {
            int32_t c = kids[kid_off[a] + it[a]++];
            vis[c] = clock++;
            stack[top++] = c;
        } else {
            fin[a] = clock++;
            --top;
        }
    }
    /* 3. flows along the BFS path of every node */
    for (int64_t u = 0; u < n; ++u) {
        int64_t s1 = 0, s2 = 0;
        for (int32_t e1 = (int32_t)u; e1 != root; e1 = bfs_par[e1]) {
            int32_t e2 = bfs_par[e1];
            if (next[e1] == e2 && vis[e1] <= vis[u] && fin[u] <= fin[e1]) {
                s1 += 1;
                s2 += ps[e1];
            }
            if (e2 != root && next[e2] == e1 && vis[e2] <= vis[u] && fin[u] <= fin[e2]) {
                s1 -= 1;
                s2 -= ps[e2];
            }
        }
        x1[u] = s1;
        x2[u] = s2;
    }
}

/*
 * SpanTree estimators over Wilson samples [sample_begin, sample_begin +
 * n_samples) (the same trees as oracle_wilson draws for these indices):
 *   kind 1 (Alg. 1): X1[u] += x1[u], X2[u] += x2[u] with w = 1 ([n] each);
 *   kind 2 (Alg. 3): per sample, s1[s] = sum_u d_u x1[u] and
 *                    s2[s] = sum_u d_u x2[u] with w = d ([n_samples] each).
 * Returns 0, -1 on allocation failure, -2 if the graph is not connected.
 */
int32_t oracle_spantree(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                        uint64_t seed, uint32_t stream, uint64_t qid,
                        int64_t sample_begin, int64_t n_samples, int32_t kind,
                        int64_t *X1, int64_t *X2, int64_t *s1, int64_t *s2, int32_t n_threads) {
    int32_t *bfs_par = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *wt = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!bfs_par || !wt) { free(bfs_par); free(wt); return -1; }
    if (oracle_bfs_tree(n, rp, col, root, bfs_par) != n) { free(bfs_par); free(wt); return -2; }
    for (int64_t u = 0; u < n; ++u) wt[u] = kind == 2 ? rp[u + 1] - rp[u] : 1;
    if (kind == 1) for (int64_t u = 0; u < n; ++u) { X1[u] = 0; X2[u] = 0; }
    int32_t status = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads)
#endif
    {
        uint8_t *intree = (uint8_t *)malloc((size_t)n);
        int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *draws = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int64_t *ps = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        int64_t *x1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        int64_t *x2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        int32_t *scr = (int32_t *)malloc(sizeof(int32_t) * 5 * (size_t)n);
        int64_t *koff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t *A1 = kind == 1 ? (int64_t *)calloc((size_t)n, sizeof(int64_t)) : NULL;
        int64_t *A2 = kind == 1 ? (int64_t *)calloc((size_t)n, sizeof(int64_t)) : NULL;
        if (!intree || !next || !draws || !ps || !x1 || !x2 || !scr || !koff || (kind == 1 && (!A1 || !A2))) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            status = -1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int64_t s = 0; s < n_samples; ++s) {
                draw_ctx dc;
                memset(&dc, 0, sizeof dc);
                dc.rp = rp; dc.col = col; dc.k0 = seed; dc.k1 = make_key1(stream, root);
                dc.c0 = (uint64_t)(sample_begin + s); dc.qid = qid;
                wilson_sample(n, root, &dc, NULL, 0, intree, next, draws, NULL, 0, NULL);
                oracle_spantree_tree(n, next, root, bfs_par, wt, ps, x1, x2, scr, koff);
                if (kind == 1) {
                    for (int64_t u = 0; u < n; ++u) { A1[u] += x1[u]; A2[u] += x2[u]; }
                } else {
                    int64_t a = 0, b = 0;
                    for (int64_t u = 0; u < n; ++u) { a += wt[u] * x1[u]; b += wt[u] * x2[u]; }
                    s1[s] = a;
                    s2[s] = b;
                }
            }
            if (kind == 1) {
#ifdef _OPENMP
#pragma omp critical(oracle_spantree)
#endif
                for (int64_t u = 0; u < n; ++u) { X1[u] += A1[u]; X2[u] += A2[u]; }
            }
        }
        free(intree); free(next); free(draws); free(ps); free(x1); free(x2); free(scr); free(koff);
        free(A1); free(A2);
    }
    free(bfs_par); free(wt);
    return status;
}

/*
 * Loop-included paths of Wilson samples [sample_begin, sample_begin +
 * n_paths) of an omega_total-sample run (Sec. 3.4): path i starts where
 * absorbed walk i of kind tag starts (tag 1 uniform over V, tag 2 stationary)
 * and follows the bottom entries of sample i's stacks until the root.  By the
 * loop-erased-walk lemma (Sec. 3.4) it is distributed as a v-absorbed walk
 * from its start, so its departures estimate the same quantities as Alg. 2's
 * and Alg. 4's walks, without fresh draws.  Y2 ([B][n], may be NULL) gets
 * the departures per node in block floor(i*B/omega_total); len_per_path
 * ([n_paths], may be NULL) the number of departures.  Returns 0, -1 on
 * allocation failure.
 */
int32_t oracle_loop_included(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                             uint64_t seed, uint32_t stream, uint64_t qid, int32_t tag,
                             int64_t sample_begin, int64_t n_paths, int64_t omega_total, int32_t B,
                             int64_t *Y2, int64_t *len_per_path, int32_t n_threads) {
    if (B < 1) B = 1;
    const uint64_t k0 = seed, k1 = make_key1(stream, root);
    const int64_t nnz = rp[n];
    int32_t status = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads)
#endif
    {
        int64_t *pos = (int64_t *)calloc((size_t)n, sizeof(int64_t));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!pos || !touched) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            status = -1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
            for (int64_t q = 0; q < n_paths; ++q) {
                const int64_t i = sample_begin + q;
                const uint64_t x0 = walk_draw(k0, k1, (uint64_t)tag, (uint64_t)i, 0, 0, qid);
                int32_t u;
                if (tag == 1) u = (int32_t)oracle_map_below(x0, (uint64_t)n);
                else if (nnz > 0) u = col[oracle_map_below(x0, (uint64_t)nnz)];
                else u = root;
                draw_ctx dc;
                memset(&dc, 0, sizeof dc);
                dc.rp = rp; dc.col = col; dc.k0 = k0; dc.k1 = k1; dc.c0 = (uint64_t)i; dc.qid = qid;
                const int64_t b = (int64_t)(((__int128)i * B) / omega_total);
                int64_t len = 0, nt = 0;
                while (u != root) {
                    if (pos[u] == 0) touched[nt++] = u;
                    const int32_t w = stack_entry(&dc, u, pos[u]);
                    pos[u] += 1;
                    if (Y2) {
#ifdef _OPENMP
#pragma omp atomic
#endif
                        Y2[b * n + u] += 1;
                    }
                    ++len;
                    u = w;
                }
                for (int64_t t = 0; t < nt; ++t) pos[touched[t]] = 0;
                if (len_per_path) len_per_path[q] = len;
            }
        }
        free(pos); free(touched);
    }
    return status;
}

/* ------------------------------------------------------------ node pairs */
/*
 * Loop-included paths from given nodes (Sec. 3.4, the loop-erased-walk
 * interpretation of L_v^{-1}): (L_v^{-1})_su is the expected number of times
 * u occurs (u != v) on the path from s through the stacks of one Wilson
 * sample, divided by d_u.  With that, the resistance of Sec. 2 is
 * r(s,t) = (L_v^{-1})_ss + (L_v^{-1})_tt - 2 (L_v^{-1})_st (grounding at v
 * leaves resistances unchanged; row and column v of the grounded inverse are
 * zero).
 *
 * For sample i in [sample_begin, sample_begin + n_samples) and pair j the path
 * from s_j and the path from t_j are run through the stacks of sample i, each
 * with its own departure counts starting at zero, so each is distributed as a
 * v-absorbed walk from its start.  Block b = floor(i*B/omega_total) of
 * V ([B][n_pairs][4]) gets:
 *   [0] departures from s_j on the path from s_j,
 *   [1] departures from t_j on the path from s_j,
 *   [2] departures from t_j on the path from t_j,
 *   [3] departures from s_j on the path from t_j.
 */
int32_t oracle_pair_paths(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                          uint64_t seed, uint32_t stream, uint64_t qid,
                          int64_t sample_begin, int64_t n_samples, int64_t omega_total, int32_t B,
                          int64_t n_pairs, const int32_t *s, const int32_t *t, int64_t *V,
                          int32_t n_threads) {
    if (B < 1) B = 1;
    const uint64_t k0 = seed, k1 = make_key1(stream, root);
    int32_t status = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads)
#endif
    {
        int64_t *pos = (int64_t *)calloc((size_t)n, sizeof(int64_t));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!pos || !touched) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            status = -1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
            for (int64_t q = 0; q < n_samples; ++q) {
                const int64_t i = sample_begin + q;
                const int64_t b = (int64_t)(((__int128)i * B) / omega_total);
                draw_ctx dc;
                memset(&dc, 0, sizeof dc);
                dc.rp = rp; dc.col = col; dc.k0 = k0; dc.k1 = k1; dc.c0 = (uint64_t)i; dc.qid = qid;
                for (int64_t j = 0; j < n_pairs; ++j) {
                    for (int side = 0; side < 2; ++side) {
                        const int32_t from = side ? t[j] : s[j];
                        const int32_t other = side ? s[j] : t[j];
                        int64_t nt = 0;
                        int32_t u = from;
                        while (u != root) {
                            if (pos[u] == 0) touched[nt++] = u;
                            const int32_t w = stack_entry(&dc, u, pos[u]);
                            pos[u] += 1;
                            u = w;
                        }
                        /* departures from the start node and from the other node */
                        const int64_t here = (from == root) ? 0 : pos[from];
                        const int64_t there = (other == root) ? 0 : pos[other];
                        int64_t *row = V + (b * n_pairs + j) * 4;
#ifdef _OPENMP
#pragma omp atomic
#endif
                        row[side ? 2 : 0] += here;
#ifdef _OPENMP
#pragma omp atomic
#endif
                        row[side ? 3 : 1] += there;
                        for (int64_t k = 0; k < nt; ++k) pos[touched[k]] = 0;
                    }
                }
            }
        }
        free(pos); free(touched);
    }
    return status;
}

/*
 * Whole rows of L_v^{-1} from loop-included paths (Sec. 3.4): for sample i in
 * [sample_begin, sample_begin + n_samples) and source j, the path from s_j
 * through the stacks of sample i; every departure from a node u adds one to
 * Y[b][j][u] ([B][n_sources][n], block b = floor(i*B/omega_total)).  Then
 * (L_v^{-1})_{s_j u} is the expectation of Y[.][j][u] / d_u per sample.
 */
int32_t oracle_lv_rows(int64_t n, const int64_t *rp, const int32_t *col, int32_t root,
                       uint64_t seed, uint32_t stream, uint64_t qid,
                       int64_t sample_begin, int64_t n_samples, int64_t omega_total, int32_t B,
                       int64_t n_sources, const int32_t *src, int64_t *Y, int32_t n_threads) {
    if (B < 1) B = 1;
    const uint64_t k0 = seed, k1 = make_key1(stream, root);
    int32_t status = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel num_threads(n_threads)
#endif
    {
        int64_t *pos = (int64_t *)calloc((size_t)n, sizeof(int64_t));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!pos || !touched) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            status = -1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
            for (int64_t q = 0; q < n_samples; ++q) {
                const int64_t i = sample_begin + q;
                const int64_t b = (int64_t)(((__int128)i * B) / omega_total);
                draw_ctx dc;
                memset(&dc, 0, sizeof dc);
                dc.rp = rp; dc.col = col; dc.k0 = k0; dc.k1 = k1; dc.c0 = (uint64_t)i; dc.qid = qid;
                for (int64_t j = 0; j < n_sources; ++j) {
                    int64_t *row = Y + (b * n_sources + j) * n;
                    int64_t nt = 0;
                    int32_t u = src[j];
                    while (u != root) {
                        if (pos[u] == 0) touched[nt++] = u;
                        const int32_t w = stack_entry(&dc, u, pos[u]);
                        pos[u] += 1;
#ifdef _OPENMP
#pragma omp atomic
#endif
                        row[u] += 1;
                        u = w;
                    }
                    for (int64_t k = 0; k < nt; ++k) pos[touched[k]] = 0;
                }
            }
        }
        free(pos); free(touched);
    }
    return status;
}
