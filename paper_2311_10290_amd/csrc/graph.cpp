// Host-side graph ingest: raw undirected edge list -> simple connected CSR
// (the input the paper's methods assume, Sec. 2).  Steps:
//   1. degrees of both orientations of every non-loop pair, row offsets;
//   2. each pair scattered into both rows;
//   3. every row sorted and its duplicates dropped (rows split over threads);
//   4. connected components by breadth-first search from the smallest
//      unlabelled id;
//   5. not connected: keep the largest component (ties: the one holding the
//      smallest id) and renumber its nodes by ascending original id, or fail;
//   6. optionally number the kept nodes by decreasing degree instead, ties by
//      increasing original id.  Hubs then share state lines and the rows of
//      nodes of equal degree lie side by side, which is where the walkers
//      start one after another.
// Neighbours come out sorted ascending (in the final numbering).
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "lap_host.h"

namespace lap {

// Runs f(lo, hi) over [0, rows) split into contiguous ranges of about equal
// weight (weights given by the row offsets rp), one range per thread.
template <class F>
static void for_row_ranges(int64_t rows, const std::vector<int64_t> &rp, F f) {
    const int64_t total = rp[rows];
    int64_t T = (int64_t)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (total < ((int64_t)1 << 20)) T = 1;
    std::vector<std::thread> th;
    int64_t lo = 0;
    for (int64_t t = 0; t < T && lo < rows; ++t) {
        const int64_t goal = total * (t + 1) / T;
        int64_t hi = (t == T - 1) ? rows : (int64_t)(std::upper_bound(rp.begin(), rp.begin() + rows + 1, goal) - rp.begin()) - 1;
        hi = std::max(hi, lo + 1);
        hi = std::min(hi, rows);
        if (t == T - 1) hi = rows;
        th.emplace_back(f, lo, hi);
        lo = hi;
    }
    for (auto &x : th) x.join();
}

int build_host_csr(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst, bool keep_lcc,
                   HostCSR &out, std::string &err, bool degree_order) {
    if (n < 1 || n >= (int64_t)1 << 31) {
        err = "n must be in [1, 2^31)";
        return LAP_EINVAL;
    }
    if (n_edges < 0 || (n_edges > 0 && (!src || !dst))) {
        err = "bad edge arrays";
        return LAP_EINVAL;
    }
    // Edges are split into T contiguous chunks, one per thread.  Each thread
    // counts its chunk's row entries, then writes them into its own slots of
    // every row (slot ranges come from the per-thread counts), so the random
    // writes of the scatter run on all threads.
    const int64_t hw = (int64_t)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    int64_t T = std::max<int64_t>(1, std::min<int64_t>(hw, ((int64_t)1 << 28) / n));   // T * n counters
    if (n_edges < ((int64_t)1 << 20)) T = 1;
    std::vector<int64_t> rp;
    std::vector<uint32_t> cnt;   // [T][n] entries of thread t's chunk in row u, then its next slot offset
    std::vector<int32_t> adj;
    std::vector<int64_t> bad((size_t)T, -1);
    auto run = [&](auto f) {
        std::vector<std::thread> th;
        for (int64_t t = 0; t < T; ++t) th.emplace_back(f, t, n_edges * t / T, n_edges * (t + 1) / T);
        for (auto &x : th) x.join();
    };
    try {
        rp.assign((size_t)n + 1, 0);
        cnt.assign((size_t)(T * n), 0u);
    } catch (...) {
        err = "host allocation failed";
        return LAP_ENOMEM;
    }
    run([&](int64_t t, int64_t lo, int64_t hi) {
        uint32_t *c = cnt.data() + t * n;
        for (int64_t e = lo; e < hi; ++e) {
            const int64_t a = src[e], b = dst[e];
            if (a < 0 || a >= n || b < 0 || b >= n) {
                bad[t] = e;
                return;
            }
            if (a == b) continue;
            ++c[a];
            ++c[b];
        }
    });
    for (int64_t t = 0; t < T; ++t)
        if (bad[t] >= 0) {
            err = "edge " + std::to_string(bad[t]) + " has a node id outside [0, n)";
            return LAP_EINVAL;
        }
    // row offsets, and each thread's first slot in every row (relative to the row)
    for (int64_t u = 0; u < n; ++u) {
        uint64_t at = 0;
        for (int64_t t = 0; t < T; ++t) {
            const uint32_t c = cnt[(size_t)(t * n + u)];
            cnt[(size_t)(t * n + u)] = (uint32_t)at;
            at += c;
        }
        if (at > 0xffffffffull) {
            err = "node " + std::to_string(u) + " has 2^32 or more edge entries";
            return LAP_EINVAL;
        }
        rp[u + 1] = rp[u] + (int64_t)at;
    }
    try {
        adj.resize((size_t)rp[n]);
    } catch (...) {
        err = "host allocation failed";
        return LAP_ENOMEM;
    }
    run([&](int64_t t, int64_t lo, int64_t hi) {
        uint32_t *c = cnt.data() + t * n;
        for (int64_t e = lo; e < hi; ++e) {
            const int32_t a = src[e], b = dst[e];
            if (a == b) continue;
            adj[(size_t)(rp[a] + c[a]++)] = b;
            adj[(size_t)(rp[b] + c[b]++)] = a;
        }
    });
    std::vector<uint32_t>().swap(cnt);
    // sort every row and drop duplicates; deg[u] = distinct neighbours
    std::vector<int64_t> deg((size_t)n, 0);
    for_row_ranges(n, rp, [&](int64_t lo, int64_t hi) {
        for (int64_t u = lo; u < hi; ++u) {
            int32_t *b = adj.data() + rp[u], *e = adj.data() + rp[u + 1];
            std::sort(b, e);
            deg[u] = std::unique(b, e) - b;
        }
    });

    // connected components: breadth-first search from the smallest unlabelled id
    std::vector<int32_t> comp((size_t)n, -1), queue;
    queue.reserve((size_t)n);
    int64_t ncomp = 0, best = -1;
    int32_t keep = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (comp[s] >= 0) continue;
        const int32_t c = (int32_t)ncomp++;
        queue.clear();
        queue.push_back((int32_t)s);
        comp[s] = c;
        for (size_t h = 0; h < queue.size(); ++h) {
            const int32_t a = queue[h];
            for (int64_t j = rp[a]; j < rp[a] + deg[a]; ++j) {
                const int32_t b = adj[(size_t)j];
                if (comp[b] < 0) {
                    comp[b] = c;
                    queue.push_back(b);
                }
            }
        }
        // components are met in order of their smallest id: the first strict
        // maximum breaks ties by smallest id
        if ((int64_t)queue.size() > best) {
            best = (int64_t)queue.size();
            keep = c;
        }
    }
    if (ncomp > 1 && !keep_lcc) {
        err = "graph has " + std::to_string(ncomp) + " connected components";
        return LAP_ENOTCONN;
    }
    std::vector<int32_t> newid((size_t)n, -1);
    out.old_ids.clear();
    for (int64_t u = 0; u < n; ++u)
        if (comp[u] == keep) out.old_ids.push_back((int32_t)u);
    if (degree_order)
        std::stable_sort(out.old_ids.begin(), out.old_ids.end(),
                         [&](int32_t a, int32_t b) { return deg[a] > deg[b]; });
    for (size_t v = 0; v < out.old_ids.size(); ++v) newid[out.old_ids[v]] = (int32_t)v;
    const int64_t n2 = (int64_t)out.old_ids.size();
    out.n = n2;
    out.rp.assign((size_t)n2 + 1, 0);
    for (int64_t v = 0; v < n2; ++v) out.rp[v + 1] = out.rp[v] + deg[out.old_ids[v]];
    out.col.resize((size_t)out.rp[n2]);
    // renumbering by ascending id keeps the order inside every row; by degree
    // the rows are sorted again
    for_row_ranges(n2, out.rp, [&](int64_t lo, int64_t hi) {
        for (int64_t v = lo; v < hi; ++v) {
            const int64_t u = out.old_ids[v];
            int32_t *o = out.col.data() + out.rp[v];
            for (int64_t j = rp[u]; j < rp[u] + deg[u]; ++j) *o++ = newid[adj[(size_t)j]];
            if (degree_order) std::sort(out.col.data() + out.rp[v], o);
        }
    });
    return LAP_OK;
}

}  // namespace lap

namespace lap {

int64_t bfs_parents(const HostCSR &g, int32_t root, std::vector<int32_t> &par) {
    const int64_t n = g.n;
    par.assign((size_t)n, -1);
    if (n == 0) return 0;
    std::vector<int32_t> queue;
    queue.reserve((size_t)n);
    std::vector<uint8_t> seen((size_t)n, 0);
    queue.push_back(root);
    seen[root] = 1;
    for (size_t h = 0; h < queue.size(); ++h) {
        const int32_t a = queue[h];
        for (int64_t j = g.rp[a]; j < g.rp[a + 1]; ++j) {
            const int32_t b = g.col[j];
            if (!seen[b]) {
                seen[b] = 1;
                par[b] = a;
                queue.push_back(b);
            }
        }
    }
    return (int64_t)queue.size();
}

}  // namespace lap
