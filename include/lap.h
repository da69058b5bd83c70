/*
 * lap.h -- C ABI of the MI355X loop-erased-walk library.
 *
 * Estimates the diagonal of the Laplacian pseudo-inverse L^dagger, electrical
 * closeness centrality and Kemeny's constant of a simple undirected connected
 * graph from Wilson loop-erased-walk samples rooted at a landmark v plus
 * v-absorbed walks, following "Scalable Algorithms for Laplacian
 * Pseudo-inverse Computation" (arXiv 2311.10290):
 *   - problem statement: Sec. 2 (input graph, L^dagger, closeness, Kemeny);
 *   - estimators: LEWalk for closeness (Alg. 2) and for Kemeny (Alg. 4);
 *   - sampling facts they rest on: Lemmas 1, 4, 5 and the Sec. 5 lemma.
 *
 * General conventions
 *   - Every function returns a lap_status; on error the outputs are left
 *     untouched and lap_last_error() returns a message (thread-local).
 *   - Host buffers are owned by the caller.  Device memory for the graph and
 *     for sampling workspace is owned by the lap_graph handle and freed by
 *     lap_graph_free().  When LAP_OUT_DEVICE is set, output pointers are
 *     device pointers owned by the caller.
 *   - Work is enqueued on the given hipStream_t (passed as void*, NULL = the
 *     null stream) and the call returns after it has completed.
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 *   - Limits: 1 <= n < 2^31; node degree < 2^24; 2m < 2^40; omega >= 1.
 *
 * Random numbers (the paper leaves the generator open).  All draws come from
 * Philox4x64-10 with key (seed, stream << 32 | root).  The k-th draw at node
 * u in Wilson sample i is the stack entry S[u][k] of Wilson's stack picture
 * (Sec. 3.4), counter (i, u, k, qid); absorbed walk i of kind t (1 = uniform
 * start, 2 = stationary start) uses counter (i | t << 56, step, 0, qid).  A
 * draw x picks index floor(x * d / 2^64) among d choices (neighbours in
 * ascending order, the n nodes, or the 2m CSR slots).  Since Wilson's stacks
 * do not depend on the order walks are run in, every execution schedule of
 * the library yields the same integer counts for the same arguments.
 */
#ifndef LAP_H
#define LAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LAP_OK = 0,
    LAP_EINVAL = -1,    /* bad argument (range, NULL, inconsistent sizes) */
    LAP_ENOTCONN = -2,  /* graph not connected and LAP_KEEP_LCC not given (L_v singular) */
    LAP_ENOMEM = -3,    /* host or device allocation failed */
    LAP_EDEVICE = -4,   /* HIP runtime error, or no device */
    LAP_ERANGE = -5,    /* a count exceeded its field (e.g. more than 2^21 - 1 draws at one
                           node in one sample) or a kernel passed its time limit */
    LAP_ECANCELED = -6  /* a served query was cancelled (lap_server_cancel) */
} lap_status;

/* ------------------------------------------------------------------ graph */

typedef struct lap_graph lap_graph;

enum { LAP_KEEP_LCC = 1, LAP_DEGREE_ORDER = 2 };

/*
 * lap_build_csr -- graph preparation (precondition of Sec. 2: simple,
 * undirected, connected).  src/dst: host arrays of n_edges node ids in
 * [0, n); each pair is an undirected edge.  Self-loops are dropped and
 * repeated pairs (in either orientation) merged.  If the result is not
 * connected: with LAP_KEEP_LCC the largest component is kept (ties: the one
 * holding the smallest id) and renumbered by ascending original id,
 * otherwise LAP_ENOTCONN.  With LAP_DEGREE_ORDER the kept nodes are then
 * numbered by decreasing degree, ties by increasing original id: the same
 * graph under a layout where hubs share cache lines and walkers started one
 * after another read neighbouring rows.  Node ids of every later call and
 * output are the final numbering; lap_graph_copy_csr's old_ids maps them back.
 * Neighbour lists are sorted ascending.  The CSR (row offsets int64[n+1],
 * columns int32[2m]) is uploaded to the device current at the call.  *out
 * receives a new handle.
 */
int lap_build_csr(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst,
                  uint32_t flags, void *hip_stream, lap_graph **out);

/* Sizes of a handle's graph (any pointer may be NULL).  max_deg_node is the
 * default landmark: the highest-degree node, lowest id on ties (Sec. 6.1). */
int lap_graph_info(const lap_graph *g, int64_t *n, int64_t *nnz, int32_t *max_deg_node,
                   int32_t *max_deg);

/* Copy the prepared graph to host arrays rp[n+1], col[nnz] and
 * old_ids[n] (original id of each node); any pointer may be NULL. */
int lap_graph_copy_csr(const lap_graph *g, int64_t *rp, int32_t *col, int32_t *old_ids);

/* Release a handle and all device memory it owns.  NULL is ignored. */
void lap_graph_free(lap_graph *g);

/* --------------------------------------------------------------- sampling */

enum {
    LAP_WANT_Y1 = 1,          /* Wilson draw counts per node, [B][n] */
    LAP_WANT_Y2_UNIFORM = 2,  /* uniform-start absorbed walks: visits per node [B][n] and lengths */
    LAP_WANT_Y2_PI = 4,       /* stationary-start absorbed walks: lengths */
    LAP_WANT_PER_SAMPLE = 8,  /* total draws of every Wilson sample */
    LAP_OUT_DEVICE = 16       /* output pointers are device pointers */
};

enum {
    LAP_MODE_AUTO = 0,        /* the wave form, or the workgroup form when too few samples to fill
                                 the device run on a large graph */
    LAP_MODE_LANE = 1,        /* one lane per sample, walks run one after another */
    LAP_MODE_WAVE = 2,        /* one wavefront per sample, 64 concurrent walkers */
    LAP_MODE_GROUP = 3,       /* one workgroup of 2, 4 or 8 wavefronts per sample, 64 walkers each */
    LAP_MODE_LDS = 4          /* one lane per sample with the CSR and the samples' state in LDS: graphs
                                 of at most 1024 nodes whose columns and state fit (lap_sample_forests,
                                 lap_sample_forests_noalloc and lap_estimate with fresh walks only;
                                 calls that read the trees back from device memory reject it).  Each
                                 sample is one sequential chain, so it pays on graphs whose walks are
                                 long (grids, paths), not where the wave form's walkers share them */
};

typedef struct {
    int64_t n_samples;     /* omega >= 1: Wilson samples, and walks of each requested kind */
    uint64_t seed;         /* Philox key word 0 */
    int32_t root;          /* landmark v; -1 = highest-degree node */
    uint32_t stream;       /* Philox key word 1 high half */
    uint64_t qid;          /* Philox counter word 3 */
    uint32_t want;         /* LAP_WANT_* bits */
    int32_t n_blocks;      /* B >= 1 contiguous sample blocks for batch-means errors */
    int64_t sample_begin;  /* index of the first sample (resuming a run) */
    int64_t n_total;       /* samples of the whole run; block of sample i = floor(i*B/n_total);
                              0 = sample_begin + n_samples */
    int32_t mode;          /* LAP_MODE_* */
    int32_t pool;          /* concurrent samples (slots); 0 = automatic (the LDS form: all samples,
                              at most 2^16 workgroups) */
    double timeout_s;      /* kernel time limit; 0 = 120 s */
    int64_t schedule;      /* wave and workgroup forms: the start scan begins at node (schedule mod n)
                              and wraps; counts do not depend on it (a knob for schedule-randomised tests) */
    int32_t group;         /* workgroup form: wavefronts per sample (2, 4 or 8); 0 = automatic */
    int32_t walks;         /* lap_estimate only: where the v-absorbed walk counts come from.
                              LAP_WALKS_FRESH (0): fresh walks with their own draws (Alg. 2, Alg. 4).
                              LAP_WALKS_LOOP (1): the loop-included paths of the same Wilson samples,
                              started like the fresh walks (Sec. 3.4: each path has the law of a
                              v-absorbed walk, so the estimates stay unbiased; sharing the samples'
                              stacks correlates them with the draw counts and shrinks the variance
                              of both estimators).  Samples then run in rounds of the state slots,
                              each round followed by its paths. */
} lap_sample_args;

enum { LAP_WALKS_FRESH = 0, LAP_WALKS_LOOP = 1 };

typedef struct {
    int64_t *y1;             /* [B][n] Wilson draws per node (sum over samples), or NULL */
    int64_t *y2;             /* [B][n] departures per node of uniform-start walks, or NULL */
    int64_t *y1_per_sample;  /* [n_samples] total draws of each Wilson sample, or NULL */
    int64_t *y2len_uniform;  /* [n_samples] length of each uniform-start walk, or NULL */
    int64_t *y2len_pi;       /* [n_samples] length of each stationary-start walk, or NULL */
    const int64_t *keep_idx; /* [n_keep] absolute sample indices to export (host array) */
    int64_t n_keep;          /* <= 64 */
    int32_t *next;           /* [n_keep][n] tree parent of each node (-1 at the root), or NULL */
    int32_t *draws;          /* [n_keep][n] draws at each node, or NULL */
} lap_counts;

/*
 * lap_sample_forests -- the integer core of Alg. 2 / Alg. 4.
 * Runs Wilson samples sample_begin .. sample_begin+n_samples-1 rooted at v
 * (Sec. 3.4) when LAP_WANT_Y1 or LAP_WANT_PER_SAMPLE or n_keep > 0, and the
 * requested absorbed walks with the same indices.  Counts are exact int64;
 * departures from a node are counted at every draw, the final arrival at the
 * tree (or at v) is not.  Outputs not requested may be NULL.
 */
int lap_sample_forests(lap_graph *g, const lap_sample_args *a, lap_counts *out, void *hip_stream);

/*
 * lap_sample_forests_noalloc -- lap_sample_forests for callers that cannot
 * allocate device memory: code under HIP graph capture, serving loops with a
 * fixed device footprint, harnesses that forbid hipMalloc.  The call makes no
 * hipMalloc or hipFree and calls no allocating library routine.
 *   - Same arguments and the same counts as lap_sample_forests, except that
 *     every output array in *out must be caller-owned DEVICE memory and a->want
 *     must include LAP_OUT_DEVICE (else LAP_EINVAL).  keep_idx stays a host
 *     array.  Absorbed walks run on the caller's stream after one another,
 *     not on an auxiliary stream.
 *   - Scratch (error word, statistics, block counts, slot epochs, walk state)
 *     is one fixed 64 MiB device array per GPU, held until the process ends
 *     and cleared by each call.  Concurrent samples are capped so that
 *     slots x n state words fit it; results do not depend on the cap.
 *   - Limits: n_blocks <= 4096 and, when Wilson samples are requested,
 *     n <= 8,384,446 nodes; beyond them LAP_ERANGE and nothing runs.
 *   - Calls that overlap on one GPU (from several host threads, or on several
 *     streams) share that scratch and race: serialise them.
 *   - The call is synchronous on hip_stream and must run on the device the
 *     graph was built on.
 */
int lap_sample_forests_noalloc(lap_graph *g, const lap_sample_args *a, lap_counts *out, void *hip_stream);

/* ------------------------------------------------------------- estimators */

typedef struct {
    double *diag;        /* [n] estimate of diag(L^dagger) (Alg. 2 output), or NULL */
    double *diag_se;     /* [n] batch-means standard error (needs B >= 2), or NULL */
    double *lv_diag;     /* [n] estimate of (L_v^{-1})_uu, 0 at v, or NULL */
    double *closeness;   /* [n] c(u) = (n-1)/(Tr + n diag_u) (Sec. 2), or NULL */
    double *trace;       /* [1] Tr(L^dagger) estimate (Kirchhoff index / n), or NULL */
    double *kemeny;      /* [1] Kemeny's constant (Alg. 4), or NULL */
    double *kemeny_se;   /* [1] its standard error from per-sample differences, or NULL */
    double *kirchhoff;   /* [1] Kirchhoff index n * Tr(L^dagger) = sum over pairs of r(s,t), or NULL */
    double *rw_betweenness; /* [n] 1/n + Tr/((n-1)(Tr + n diag_u)) (end of Sec. 5), or NULL */
} lap_estimates;

/*
 * lap_estimate -- one pass of the hot path: omega Wilson samples, omega
 * uniform-start absorbed walks if any of diag/diag_se/closeness/trace is
 * requested, omega stationary-start walks if kemeny is requested, and the
 * FP64 assembly on the device:
 *   diag_u = (Y1_u - 2 Y2_u) / (omega d_u) + (1/n) sum_w Y2_w / (omega d_w)   (Alg. 2)
 *   kappa  = (sum_i y1_i - sum_i len_i) / omega                               (Alg. 4)
 * Output pointers are host pointers unless LAP_OUT_DEVICE is set in a->want.
 */
int lap_estimate(lap_graph *g, const lap_sample_args *a, lap_estimates *out, void *hip_stream);

/* Convenience forms of lap_estimate with default arguments (automatic mode,
 * stream 0, qid 0, B = 64 when se is requested).  root = -1 picks the
 * highest-degree node.  Host outputs. */
int lap_diag_Ldagger(lap_graph *g, int32_t root, int64_t omega, uint64_t seed, double *diag,
                     double *se, void *hip_stream);
int lap_ecc(lap_graph *g, int32_t root, int64_t omega, uint64_t seed, double *c,
            double *trace_Ldagger, void *hip_stream);
int lap_kemeny(lap_graph *g, int32_t root, int64_t omega, uint64_t seed, double *kappa,
               double *se, void *hip_stream);

/* --------------------------------------------------------------- batching */

/*
 * Many independent estimation jobs in one persistent launch.  Each job is
 * exactly the computation of one lap_estimate call on its own graph (omega
 * Wilson samples, omega uniform-start and omega stationary-start absorbed
 * walks, FP64 assembly; Alg. 2 and Alg. 4) with B = 1, and draws the same
 * Philox stream, so its counts equal those of lap_sample_forests with the
 * same (seed, stream, qid, root, omega) bit for bit.  The graphs live in one
 * device arena; resident wavefronts take work items (a chunk of Wilson
 * samples of one job, or 64 walks of one job) from one atomic counter.
 */
typedef struct lap_batch lap_batch;

typedef struct {
    int64_t n;               /* nodes of the raw edge list */
    int64_t n_edges;
    const int32_t *src;      /* host arrays, as for lap_build_csr */
    const int32_t *dst;
    uint32_t flags;          /* LAP_KEEP_LCC | LAP_DEGREE_ORDER */
    int32_t root;            /* -1 = highest-degree node */
    int64_t n_samples;       /* omega >= 1 */
    uint64_t seed;
    uint32_t stream;
    uint64_t qid;
} lap_batch_job;

typedef struct {
    int32_t pool;            /* resident wavefronts; 0 = 16 per compute unit */
    int32_t chunk_nodes;     /* Wilson samples per work item ~ chunk_nodes / n; 0 = 2^17 */
    int32_t use_graph;       /* capture the run in a hipGraph once and replay it */
    double timeout_s;        /* kernel time limit; 0 = 300 s */
} lap_batch_tuning;

typedef struct {
    int64_t *y1;             /* [n] Wilson draws per node, or NULL */
    int64_t *y2;             /* [n] uniform-start walk departures per node, or NULL */
    int64_t *y1_per_sample;  /* [omega], or NULL */
    int64_t *y2len_uniform;  /* [omega], or NULL */
    int64_t *y2len_pi;       /* [omega], or NULL */
    double *diag;            /* [n] diag(L^dagger) estimate, or NULL */
    double *closeness;       /* [n], or NULL */
    double *trace;           /* [1], or NULL */
    double *kemeny;          /* [1], or NULL */
    double *kemeny_se;       /* [1], or NULL */
} lap_batch_out;

/* Prepare every job's graph (as lap_build_csr) into one device arena. */
int lap_batch_create(const lap_batch_job *jobs, int32_t n_jobs, void *hip_stream, lap_batch **out);
/* Prepared size and landmark of one job. */
int lap_batch_job_info(const lap_batch *b, int32_t job, int64_t *n, int64_t *nnz, int32_t *root);
/* Run all jobs (t may be NULL for defaults); synchronous on hip_stream.  With
 * use_graph the launch sequence (clears, persistent kernel, assembly) is
 * captured once per tuning on an internal stream and replayed. */
int lap_batch_run(lap_batch *b, const lap_batch_tuning *t, void *hip_stream);
/* Time a grid of pool sizes (8, 16, 24 waves per CU) and chunk sizes (2^15,
 * 2^17 node-samples per Wilson item) on the whole batch, after one untimed warm-up run, and return
 * (with use_graph set) the largest pool among the tunings within 3% of the
 * fastest, at its fastest chunk size; *best_ms is that tuning's time.  When
 * the batch is a probe subset of a larger one, the larger pool is the safer
 * pick there. */
int lap_batch_autotune(lap_batch *b, lap_batch_tuning *best, double *best_ms, void *hip_stream);
/* Copy one job's results of the last run to host buffers (NULL = skip). */
int lap_batch_result(const lap_batch *b, int32_t job, lap_batch_out *out);
/* Walk steps and trees of the last run, all jobs together. */
int lap_batch_stats(const lap_batch *b, int64_t *wilson_steps, int64_t *absorbed_steps, int64_t *trees);
void lap_batch_free(lap_batch *b);

/*
 * lap_landmark_traces -- the landmark study (Sec. 6.2, the effect of the
 * landmark; Table 1 reports Tr((I-P_v)^{-1})/n): for each roots[j], omega
 * Wilson samples rooted there (seed, stream 0, qid 0: the same draws as
 * lap_sample_forests with that root); trace[j] receives their mean total
 * draws, an unbiased estimate of Tr((I-P_v)^{-1}) -- the expected cost of
 * one sample (Sec. 3.3) -- and trace_se[j] (may be NULL) its standard error.
 * All roots run in one persistent launch over the shared graph.
 */
int lap_landmark_traces(lap_graph *g, const int32_t *roots, int32_t n_roots, int64_t omega, uint64_t seed,
                        double *trace, double *trace_se, void *hip_stream);

/* ---------------------------------------------------------------- SpanTree */

/*
 * lap_spantree -- the per-tree sums of the SpanTree estimators (Alg. 1 for
 * diag(L^dagger) and closeness, Alg. 3 for Kemeny's constant) over the
 * Wilson trees of samples [sample_begin, sample_begin + n_samples): the same
 * trees lap_sample_forests draws for these arguments.  With T a sampled tree
 * rooted at v and the BFS path of u towards v (a BFS tree from v, neighbours
 * in ascending order), every edge (e1, e2) of that path which is a tree edge
 * lying on u's own tree path (its lower end an ancestor-or-self of u, by DFS
 * intervals) contributes the flow it carries in the direction e1 -> e2
 * (Sec. 4.1 and Sec. 5.2; the containment test as printed is reversed, see
 * the design notes):
 *   x1(u)  +1 / -1            (unit current entering at u, leaving at v);
 *   x2(u)  +/- |subtree(lower end)|            (1/n entering at every node,
 *          in units of 1/n);
 *   x2'(u) +/- degree sum of the subtree        (d_w/2m entering at every w,
 *          in units of 1/2m).
 * Outputs (int64; host memory unless a->want has LAP_OUT_DEVICE; any NULL):
 *   X1, X2 [B][n]      per block b of samples (i*B/n_total == b), the sums
 *                      of x1(u) and x2(u);
 *   s1, s2 [n_samples] per sample, sum_u d_u x1(u) and sum_u d_u x2'(u).
 * Arguments as for lap_sample_forests (mode, pool, group, schedule, seed,
 * stream, qid); want bits other than LAP_OUT_DEVICE are ignored.  The BFS
 * tree is computed on the host once per root.  Scratch: 36 bytes per node
 * per tree in flight (at most 48 GiB).  LAP_ENOTCONN for a disconnected graph.
 */
int lap_spantree(lap_graph *g, const lap_sample_args *a, int64_t *X1, int64_t *X2, int64_t *s1, int64_t *s2,
                 void *hip_stream);

/*
 * lap_spantree_estimate -- FP64 SpanTree estimates of a whole sample set
 * (sample_begin 0, n_total = n_samples): diag [n] = x1(u) - 2 x2(u) +
 * (1/n) sum_w x2(w) with x1 = X1/omega and x2 = X2/(n omega) (Alg. 1, last
 * loop); diag_se [n] by batch means over the B blocks; closeness [n] =
 * (n-1)/(Tr + n diag(u)); kemeny = mean over samples of s1 - s2/2m (Alg. 3)
 * and kemeny_se.  Any output may be NULL; host or device as above.
 */
int lap_spantree_estimate(lap_graph *g, const lap_sample_args *a, double *diag, double *diag_se, double *closeness,
                          double *kemeny, double *kemeny_se, void *hip_stream);

/*
 * lap_spantree_sample_bound -- the Hoeffding sample sizes of the SpanTree
 * analysis (Thm. 3 for Alg. 1, Thm. 4 for Alg. 3): with D the depth of the
 * BFS tree from v (the longest path a flow is sent along),
 *   kind 1 (closeness): omega >= 32 D^2 ln(2n / p_fail) / eps^2 gives
 *          |estimate - (L^dagger)_uu| <= eps for all u with probability at
 *          least 1 - p_fail;
 *   kind 2 (Kemeny):    omega >= 8 m^2 D^2 ln(2 / p_fail) / eps^2 gives
 *          |estimate - kappa| <= eps with probability at least 1 - p_fail
 *          (m undirected edges).
 * root = -1: the max-degree node.  Writes the bound, rounded up, to *omega
 * (a double: the bounds outgrow 64-bit integers quickly) and D to *depth
 * (either may be NULL).  Host only: no device work.
 */
int lap_spantree_sample_bound(const lap_graph *g, int32_t root, int32_t kind, double eps, double p_fail,
                              double *omega, int32_t *depth);

/*
 * lap_loop_included -- loop-included paths of the Wilson stacks (Sec. 3.4,
 * the loop-erased-walk interpretation of L_v^{-1}): for every sample i of a,
 * the path that starts where absorbed walk i of kind tag starts (1: uniform
 * over V, counter (i | 1<<56, 0, 0, qid); 2: stationary, (i | 2<<56, 0, 0,
 * qid)) and at its c-th departure from u moves to stack entry S_i[u][c] --
 * the same draw the sampler used -- until it reaches v.  Such a path is
 * distributed as a v-absorbed walk from its start, so its departures
 * estimate the same quantities as the walks of lap_sample_forests
 * (LAP_WANT_Y2_UNIFORM / LAP_WANT_Y2_PI) without draws of their own.
 * Outputs (int64; host unless LAP_OUT_DEVICE; either may be NULL):
 *   Y2  [B][n]        departures per node, per block of samples;
 *   len [n_samples]   departures per path.
 * Scratch: 4 bytes per node per path in flight (at most 48 GiB).
 */
int lap_loop_included(lap_graph *g, const lap_sample_args *a, int32_t tag, int64_t *Y2, int64_t *len,
                      void *hip_stream);

/*
 * lap_pair_paths -- entries of L_v^{-1} and effective resistances of node
 * pairs from loop-included paths of the Wilson stacks (Sec. 3.4, the
 * loop-erased-walk interpretation of L_v^{-1}; r(s,t) of Sec. 2, unchanged by
 * grounding at v).  For every sample i of a and pair j, the path from s_j
 * and the path from t_j through the stacks of sample i, each taking at its
 * c-th departure from u the entry S_i[u][c] (Philox counter (i, u, c, qid):
 * the sampler's own draws), until they reach v.  The departures from u of the
 * path from s, divided by d_u, estimate (L_v^{-1})_su.
 *   ps, pt  [n_pairs] node ids (host), 1 <= n_pairs <= 2^30; a node may be v
 *           (its row of the grounded inverse is zero) and s == t is allowed.
 *   check   1: run the Wilson samples too and fail with LAP_EDEVICE if a path
 *           ever uses an entry the sampler did not draw (c >= k_u; by the
 *           order independence of the stacks this never happens);
 *           0: read the same entries without running the sampler (identical
 *           results, no Wilson work).
 *   lanes   paths in flight; 0 picks up to 2^17 within 32 GiB of departure
 *           counters per lane: a 16384-word hash table on graphs of more
 *           than 16384 nodes (a path that meets more than 12288 distinct
 *           nodes is rerun with n words), n words otherwise.  A positive
 *           value caps it; the results do not depend on it.
 * Outputs (host unless LAP_OUT_DEVICE; any may be NULL):
 *   V     int64 [B][n_pairs][4] per sample block: departures from s on the
 *         path from s, from t on the path from s, from t on the path from t,
 *         from s on the path from t (exact);
 *   r     [n_pairs] (V0/d_s - V1/d_t + V2/d_t - V3/d_s) / omega over all blocks;
 *   r_se  [n_pairs] batch-means standard error of r (NaN when B == 1);
 *   lv    [n_pairs][3] (L_v^{-1})_ss, (L_v^{-1})_st, (L_v^{-1})_tt with
 *         the off-diagonal entry averaged over both orders:
 *         V0/(omega d_s), (V1/d_t + V3/d_s)/(2 omega), V2/(omega d_t).
 * Scratch: the lanes' counters (at most 32 GiB per form), 8 bytes per
 * path of a launch for the rerun queue, and the Wilson state when check is
 * 1.  Walk steps are reported by lap_last_stats as absorbed steps.
 */
int lap_pair_paths(lap_graph *g, const lap_sample_args *a, const int32_t *ps, const int32_t *pt,
                   int64_t n_pairs, int32_t check, int64_t lanes, int64_t *V, double *r, double *r_se,
                   double *lv, void *hip_stream);

/*
 * lap_lv_rows -- whole rows of L_v^{-1} from loop-included paths of the
 * Wilson stacks (Sec. 3.4, the loop-erased-walk interpretation of L_v^{-1}):
 * for every sample i of a and source j, the path from s_j through the stacks
 * of sample i, taking at its c-th departure from u the entry S_i[u][c]
 * (Philox counter (i, u, c, qid)), until it reaches v.  Every departure from
 * u adds one to the source's row at u; (L_v^{-1})_{s_j u} is its expectation
 * per sample over d_u.
 *   sources [n_sources] node ids (host), 1 <= n_sources <= 2^23; a source may
 *           be v (its row is zero).
 *   check, lanes  as for lap_pair_paths.
 * Outputs (host unless LAP_OUT_DEVICE; either may be NULL):
 *   Y     int64 [B][n_sources][n] departures per node, per sample block (exact);
 *   rows  [n_sources][n] sum over blocks of Y / (omega d_u), 0 in column v.
 * B * n_sources * n must stay within 2^33.  Scratch as for lap_pair_paths.
 */
int lap_lv_rows(lap_graph *g, const lap_sample_args *a, const int32_t *sources, int64_t n_sources,
                int32_t check, int64_t lanes, int64_t *Y, double *rows, void *hip_stream);

/* ---------------------------------------------------------------- serving */

/*
 * A request loop over one resident graph.  Query kinds:
 *   LAP_Q_CLOSENESS  c(u) from `budget` walks started at u and absorbed at v:
 *                    (L_v^{-1})_uu = E[departures from u]/d_u (Lemma 1) and
 *                    e_u^T L_v^{-1} 1 = E[sum of 1/d over departures]
 *                    (normalised-length lemma, Sec. 4.3), combined with the
 *                    cached Tr(L_v^{-1}) and 1^T L_v^{-1} 1 through the
 *                    element-wise equation for L^dagger_uu and
 *                    Tr(L^dagger) = Tr(L_v^{-1}) - 1^T L_v^{-1} 1 / n (Sec. 3.1);
 *   LAP_Q_RESISTANCE r(u,w) = (L_v^{-1})_uu + (L_v^{-1})_ww - 2 (L_v^{-1})_uw
 *                    from `budget` pairs of walks from u and from w;
 *   LAP_Q_KEMENY     Kemeny's constant from `budget` Wilson samples and
 *                    stationary-start walks (Alg. 4).
 * Query walk i (sub-stream 0 from u, 1 from w) uses counter
 * (i | 3<<56, move, sub, qid); a Kemeny query draws exactly what
 * lap_estimate with qid = the query id and omega = budget draws.  A result
 * therefore does not depend on which other queries were in flight.
 *
 * Scheduling: lap_server_submit queues a query.  lap_server_step retires
 * finished launches, admits queued queries in arrival order while their
 * result regions fit in the device result arena (arena_bytes), and starts a
 * launch on every idle stream with the active queries' next work items, one
 * per query per round (continuous batching: queries that arrive while
 * launches are running join the next launch).  With two or more streams,
 * even-numbered streams carry walk tiles and odd ones Wilson samples, so
 * short queries do not wait behind the Wilson samples of Kemeny queries.  Completed queries are
 * assembled on the host in FP64 and returned by lap_server_poll.
 */
typedef struct lap_server lap_server;

enum { LAP_Q_CLOSENESS = 0, LAP_Q_RESISTANCE = 1, LAP_Q_KEMENY = 2 };

/* the query id the server uses for its own cached global terms */
#define LAP_SERVER_GLOBAL_QID 0xFFFFFFFFFFFFFFFFull

typedef struct {
    int64_t qid;             /* >= 0; keys the query's random stream */
    int32_t kind;            /* LAP_Q_* */
    int32_t u, w;            /* node (closeness), pair (resistance) */
    int64_t budget;          /* walks, walk pairs or samples */
} lap_query;

typedef struct {
    int64_t qid;
    int32_t kind;
    int32_t status;          /* LAP_OK, or the error that stopped the query */
    double value;            /* c(u), r(u,w) or kappa */
    double se;               /* standard error of value over the query's own walks / samples.
                                For closeness it is conditional on the cached global term
                                Tr(L_v^{-1}) of lap_server_create (the only global term that
                                enters c(u)), which it treats as exact. */
    double t_submit, t_start, t_done;   /* seconds since lap_server_create */
} lap_query_result;

typedef struct {
    uint64_t seed;
    int32_t root;            /* -1 = highest-degree node */
    uint32_t stream;
    int64_t global_samples;  /* samples for the cached global terms; 0 = 256 */
    int64_t arena_bytes;     /* device memory for query results; 0 = 64 MiB */
    int32_t launches;        /* launches in flight (streams); 0 = 5 */
    int32_t waves;           /* wavefronts (Wilson state slots) per launch; 0 = 4 per CU */
    int32_t items_per_launch;/* 0 = 4096; a Wilson-only launch takes at most `waves` items */
    int32_t wilson_chunk;    /* Wilson samples per work item; 0 = 1 */
    double timeout_s;        /* kernel time limit; 0 = 300 s */
    int32_t wilson_group;    /* wavefronts per Wilson sample in Wilson launches: 1 = wave form,
                                2, 4 or 8 = workgroup form; 0 = 4 on graphs of >= 2^16 nodes, else 1 */
    int32_t wilson_slots;    /* Wilson samples per Wilson launch at most (bounds the Wilson work
                                that shares the device with walk tiles); 0 = waves */
} lap_server_config;

/* Compute the cached global terms (lap_sample_forests with qid
 * LAP_SERVER_GLOBAL_QID) and allocate the arena, the Wilson state of every
 * launch (launches * waves * n * 8 bytes) and the streams.  The graph must
 * outlive the server. */
int lap_server_create(lap_graph *g, const lap_server_config *cfg, void *hip_stream, lap_server **out);
/* Queue a query (thread-safe).  LAP_ENOMEM if its result region could never
 * fit in the arena. */
int lap_server_submit(lap_server *s, const lap_query *q);
/* Retire, admit and launch (see above); with wait != 0 first block until a
 * running launch completes. */
int lap_server_step(lap_server *s, int32_t wait);
/* Cancel a queued or running query: a queued one leaves the queue at once; a
 * running one issues no further work items, and its result region returns to
 * the arena when the items already on the device have come back.  Either way
 * lap_server_poll then returns its record with status LAP_ECANCELED and a NaN
 * value.  Other queries' results are unchanged (they draw their own keyed
 * streams).  LAP_EINVAL if no queued or running query has this id. */
int lap_server_cancel(lap_server *s, int64_t qid);
/* Move up to max completed results to out; *n_out receives their number. */
int lap_server_poll(lap_server *s, lap_query_result *out, int32_t max, int32_t *n_out);
/* Queries waiting for admission, admitted and not finished, launches running. */
int lap_server_pending(lap_server *s, int64_t *queued, int64_t *active, int64_t *inflight);
/* The cached Tr(L_v^{-1}) and 1^T L_v^{-1} 1. */
int lap_server_globals(const lap_server *s, double *trace_lv, double *sum_lv);
void lap_server_free(lap_server *s);

/* ---------------------------------------------------------------- support */

/* Message for the last error on this thread ("" if none). */
const char *lap_last_error(void);

/* Kernel timing: when enabled, every kernel launch of the library is
 * bracketed by HIP events on the stream it runs on; lap_prof_read returns
 * the accumulated milliseconds and launch count for a kernel name
 * ("wilson_wave", "wilson_lane", "wilson_group", "wilson_lds", "spantree", "loop_included",
 * "pair_paths", "pair_assemble", "lv_rows", "absorbed", "assemble",
 * "batch", "batch_assemble").  Returns
 * LAP_EINVAL for an unknown name. */
int lap_prof_enable(int on);
int lap_prof_reset(void);
int lap_prof_read(const char *kernel, double *total_ms, int64_t *launches);

/* Counters of the last lap_sample_forests / lap_estimate call: Wilson walk
 * steps (draws), absorbed-walk steps, completed trees, wave iterations,
 * deadlock pops, rescans, and summed over wave iterations the number of
 * idle walkers and of parked walkers.  Any pointer may be NULL. */
int lap_last_stats(const lap_graph *g, int64_t *wilson_steps, int64_t *absorbed_steps,
                   int64_t *trees, int64_t *iterations, int64_t *pops, int64_t *rescans,
                   int64_t *idle_lane_rounds, int64_t *parked_lane_rounds);

/* Random-gather rate of the current device, the roofline reference for the
 * walkers: memory operations per second (written to *rate) of random 8-byte
 * accesses over a working set of `bytes` (>= 1 MiB, rounded down to a power
 * of two) by `lanes` (256 .. 2^24) concurrent lanes.  mode 0: each lane issues
 * `in_flight` (1, 2, 4, 8 or 16) independent loads per round; mode 1: each lane
 * follows a dependent pointer chain through a random cyclic order of 64-byte
 * lines (in_flight must be 1, 2, 4, 8 or 16 and is ignored); mode 2: as mode 0
 * plus one random 8-byte store per round; mode 3: as mode 0 plus one store of a
 * whole random 64-byte line per round (modes 2 and 3 count loads and stores, a
 * line store once, and take plain loads only); mode 4: `in_flight` random
 * 4-byte reads per round from a 64 KiB table in LDS, rounds dependent (bytes is
 * then only checked; plain reads only).  flavor: 0 plain loads, 1 non-temporal loads, 2 relaxed atomic
 * loads at device scope, 3 at system scope.  A sweep over lanes and in_flight
 * gives each working-set tier's peak.  Allocates and frees its own buffer;
 * LAP_EINVAL on bad arguments. */
int lap_bench_gather(int64_t bytes, int64_t lanes, int32_t mode, int32_t in_flight, int32_t flavor,
                     double *rate, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LAP_H */
