// Host-side internals of the library: graph handle, workspace, ingest.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lap.h"
#include "lap_device.h"

namespace lap {

struct HostCSR {
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<int32_t> old_ids;
};

// degree_order: number the kept nodes by decreasing degree, ties by
// increasing original id (a relabelling of the same graph; old_ids maps back)
int build_host_csr(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst, bool keep_lcc,
                   HostCSR &out, std::string &err, bool degree_order = false);

// graphs whose column array has at least this many bytes also get arc
// records: every graph (with the Wilson samplers' arc form and degree
// numbering the records pay even where columns and rows stay in cache)
constexpr int64_t kArcsMinColBytes = 0;

// BFS tree of the CSR from root, neighbours in ascending order: par[u] is u's
// parent, -1 at the root.  Returns the number of nodes reached.
int64_t bfs_parents(const HostCSR &g, int32_t root, std::vector<int32_t> &par);

// Set the thread's error text and return code.
int fail(int code, const std::string &msg);

// Arguments of a sampling call, checked and resolved against the graph
// (capi.cpp): sample range, landmark, blocks, sampler form and concurrent
// sample slots.
struct Resolved {
    int64_t omega, begin, total;
    int32_t root, B, mode, group;
    int32_t lds_lanes;   // LDS lane form: samples per workgroup
    int64_t slots;
    bool wilson, y2u, y2p;
};

// reads_trees: the call reads the Wilson trees back from the state slots
// (SpanTree, loop-included paths), so the LDS lane form, which keeps its state
// in LDS only, is refused and never chosen automatically.
int resolve_args(const lap_graph *g, const lap_sample_args *a, int64_t n_keep, const int64_t *keep_idx,
                 Resolved &r, bool reads_trees = false);

// Samples per workgroup of the LDS lane form on this graph (64, 32 or 16), or
// 0 when the graph has too many nodes or its columns and state do not fit.
int32_t lds_lanes(const lap_graph *g);

// Status and error text for a device-side error word (LAP_OK when clear).
int status_from_err(const DevErr &e);

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::lap::fail(e_ == hipErrorOutOfMemory ? LAP_ENOMEM : LAP_EDEVICE,     \
                               std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

// Optional per-kernel timing: events around launches, accumulated by name
// after the caller's streams have been synchronised (lap_prof_*).
struct Timer {
    struct PendingEvent {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<PendingEvent> pending;
    bool on = false;
    Timer();
    ~Timer();
    void begin(const char *name, hipStream_t s);
    void end(hipStream_t s);
    void collect();
};

// A device allocation that only grows.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t want);
    void release();
    template <class T>
    T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace lap

// The graph handle of include/lap.h: host CSR, device CSR and the sampling
// workspace the calls reuse.
struct lap_graph {
    int device = 0;
    int n_cu = 256;
    double clock_khz = 100000.0;
    int64_t lds_per_block = 65536;   // LDS bytes a workgroup may use
    lap::HostCSR csr;
    int32_t max_deg_node = 0, max_deg = 0;
    lap::DevBuf rp, nbr, col, arcs;   // arcs: per column entry {target, its adjacency record}, large graphs only
    // sampling workspace
    lap::DevBuf state, epoch;
    int64_t state_slots = 0;
    bool state_dirty = false;
    lap::DevBuf y1, y2, y1s, len_u, len_p, keep_next, keep_draws, err, stats;
    lap::DevBuf asm_partial, asm_sums, asm_trace, est_out, blkcount;
    // SpanTree workspace: BFS parents for bfs_root, per-tree scratch, sums
    int32_t bfs_root = -1;
    lap::DevBuf bfs_par, span64, span32, span_x, span_s;
    lap::DevBuf loop_cnt, loop_y2, loop_len;   // loop-included paths
    // loop-included paths from node pairs: per-lane counter words and last
    // tags (dense and hashed forms; lanes set up so far), queue, counters
    lap::DevBuf pair_cnt, pair_cnt_tags, pair_tbl, pair_tbl_tags, pair_queue, pair_next, pair_ids, pair_v, pair_out;
    lap::DevBuf pair_rows, pair_rows_out;   // lap_lv_rows: counts and rows
    int64_t pair_cnt_lanes = 0, pair_tbl_lanes = 0;
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int64_t last_stats[lap::kNumStats] = {0};
    ~lap_graph() {
        lap::DevBuf *bufs[] = {&rp, &nbr, &col, &arcs, &state, &epoch, &y1, &y2, &y1s, &len_u, &len_p, &keep_next,
                          &keep_draws, &err, &stats, &asm_partial, &asm_sums, &asm_trace, &est_out, &blkcount,
                          &bfs_par, &span64, &span32, &span_x, &span_s, &loop_cnt, &loop_y2, &loop_len,
                          &pair_cnt, &pair_cnt_tags, &pair_tbl, &pair_tbl_tags, &pair_queue, &pair_next,
                          &pair_ids, &pair_v, &pair_out, &pair_rows, &pair_rows_out};
        for (lap::DevBuf *b : bufs) b->release();
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (aux) (void)hipStreamDestroy(aux);
    }
};


