// Parameter blocks of the kernels beyond the Wilson samplers: the batched
// launch, the serving launch, the SpanTree pass, the loop-included paths (from
// absorbed-walk starts and from node pairs) and the SpanTree assembly.
#pragma once

#include "lap_device.h"

namespace lap {

// ------------------------------------------------------------ batched jobs
struct BatchJobDev {
    int64_t node_off;      // first node of the job in the arena (nbr, y1, y2, diag, closeness)
    int64_t col_off;       // first column entry of the job in the arena
    int64_t n, nnz, omega;
    int64_t sample_off;    // first entry of the job in the per-sample arrays
    int32_t root;
    int32_t pad;
    uint64_t k0, k1, qid;  // Philox key and counter word 3
};

struct BatchItem {
    int32_t job;
    int32_t kind;          // 0 Wilson samples, 1 uniform-start walks, 2 stationary-start walks
    int64_t first, count;
};

struct BatchParams {
    const BatchJobDev *jobs;
    const BatchItem *items;
    int64_t n_items;
    unsigned long long *counter;
    const uint64_t *nbr;   // arena, offsets relative to each job's col_off
    const int32_t *col;    // arena, job-local node ids
    uint64_t *state;       // [waves][max_n]
    int64_t max_n;
    unsigned long long *y1, *y2;          // [sum n]
    int64_t *y1s, *len_u, *len_p;         // [sum omega]
    double *diag, *closeness;             // [sum n]
    double *trace, *kemeny, *kemeny_se;   // [jobs]
    unsigned long long *stats;
    DevErr *err;
    uint64_t deadline;
};

// ------------------------------------------------------------ serving
struct ServeItem {
    int32_t kind;          // 0 Wilson samples, 2 stationary-start walks, 3 closeness walks, 4 resistance pairs
    int32_t count;         // samples or walks in this item (<= 64 for walk items)
    int64_t first;         // first sample / walk index within the query
    int64_t budget;        // the query's sample / walk budget (stride of its result arrays)
    int64_t qid;           // query id: Philox counter word 3
    int32_t u, w;          // query nodes
    int64_t out_off;       // the query's region in the result arena (8-byte words)
};

struct ServeParams {
    int64_t n, nnz;
    const uint64_t *nbr;
    const int32_t *col;
    const ulonglong2 *arcs;   // or null
    int32_t root;
    uint64_t k0, k1;
    const ServeItem *items;
    int64_t n_items;
    unsigned long long *counter;
    uint64_t *state;       // [slots][n]
    uint32_t *slot_epoch;  // [slots]
    int64_t slot_base;     // this launch's first slot
    uint64_t *arena;       // result words
    unsigned long long *stats;
    DevErr *err;
    uint64_t deadline;
};

// SpanTree pass over the trees left in the Wilson state slots (spantree.hip)
constexpr int64_t kSpanInt64PerNode = 3;   // scratch per node per tree: 3 int64 + 3 int32
constexpr int64_t kSpanInt32PerNode = 3;

struct SpanParams {
    int64_t n;
    const uint64_t *nbr;
    int32_t root;
    const uint64_t *state;         // [slots][n]: slot s holds the tree of sample sample_begin + s
    int64_t n_trees;
    int64_t sample_begin, n_total;
    int32_t n_blocks;
    const int32_t *bfs_par;        // [n] BFS parents from the root (-1 at the root)
    int64_t *scratch64;            // [n_trees][3][n]
    int32_t *scratch32;            // [n_trees][3][n]
    unsigned long long *X1, *X2;   // [B][n] unit-flow and path-support sums, or null
    long long *s1, *s2;            // [n_trees] Kemeny terms of this launch's samples, or null
    DevErr *err;
};

// Loop-included paths over the trees left in the Wilson state slots (loops.hip)
struct LoopParams {
    int64_t n, nnz;
    const uint64_t *nbr;
    const int32_t *col;
    int32_t root;
    uint64_t k0, k1, qid;
    uint32_t tag;                  // start like absorbed walk kind 1 (uniform) or 2 (stationary)
    const uint64_t *state;         // [slots][n]
    const uint32_t *slot_epoch;    // [slots]
    int32_t *cnt;                  // [n_paths][n] departures so far, zero before the launch
    int64_t n_paths, sample_begin, n_total;
    int32_t n_blocks;
    unsigned long long *y2;        // [B][n] or null
    int64_t *len_out;              // [n_paths] of this launch, or null
    unsigned long long *stats;     // path steps are added to the absorbed-step count, or null
    DevErr *err;
    uint64_t deadline;
};

// Loop-included paths from node pairs, or from sources for whole rows of L_v^{-1},
// over the stacks of the launch's samples (loops.hip)
struct PairParams {
    int64_t n;
    const uint64_t *nbr;
    const int32_t *col;
    int32_t root;
    uint64_t k0, k1, qid;
    const uint64_t *state;         // [samples][n] Wilson trees of the launch's samples, or null (no check)
    const uint32_t *slot_epoch;    // [samples], with state
    const int32_t *ps, *pt;        // [n_pairs]
    int64_t n_pairs;
    uint64_t *cnt;                 // dense form: [n_lanes][n] tag << 32 | count
    uint64_t *tbl;                 // hashed form: [n_lanes][2^hash_log2] node | tag << 32 | count << 48
    int32_t hash_log2, hash_limit; // table size, and distinct nodes a path may meet in it
    uint32_t *lane_tag;            // [n_lanes] last tag each lane used in its words
    int64_t n_lanes;
    int64_t n_items;               // items slot * 2 n_pairs + q of the launch (when queue_in is null)
    const unsigned long long *queue_in;      // or the items to run: [*queue_in_len]
    const unsigned long long *queue_in_len;
    unsigned long long *queue_out;           // hashed form: items left to the dense form
    unsigned long long *queue_out_len;
    unsigned long long *next;      // [n_parts * 16] item counters, zero before the launch
    int32_t n_parts;
    int64_t sample_begin, n_total;
    int32_t n_blocks;
    unsigned long long *V;         // [B][n_pairs][4]
    unsigned long long *rows;      // rows form: [B][n_pairs][n] departures per node of the paths from ps
                                   // (one path per source; pt and V unused), or null
    unsigned long long *stats;
    DevErr *err;
    uint64_t deadline;
};

struct PairAsmParams {
    const uint64_t *nbr;
    const int32_t *ps, *pt;
    int64_t n_pairs, omega;
    int32_t B;
    const unsigned long long *V;   // [B][n_pairs][4]
    double *r, *r_se, *lv;         // [n_pairs], [n_pairs], [n_pairs][3]; any may be null
};

struct SpanAsmParams {
    int64_t n, omega, two_m;
    int32_t B;
    const unsigned long long *X1, *X2;   // [B][n]
    const int64_t *blk_n;                // [B] samples per block
    long long *blk_sum;                  // [B] scratch
    const long long *s1, *s2;            // [omega]
    double *diag, *diag_se, *closeness, *trace, *kemeny, *kemeny_se;   // any may be null (diag needed for the rest)
    double *part;                        // [n_parts] per-workgroup partial traces
    int64_t n_parts;
};

}  // namespace lap
