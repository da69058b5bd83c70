// Host-side graph ingest: raw undirected edge list -> simple connected CSR
// (the input the paper's methods assume, Sec. 2).  Steps:
//   1. both orientations of every non-loop pair become 64-bit keys row*n+col;
//   2. LSD radix sort of the keys, adjacent duplicates dropped;
//   3. connected components by union-find over the kept pairs;
//   4. not connected: keep the largest component (ties: the one holding the
//      smallest id) and renumber its nodes by ascending original id, or fail;
//   5. row offsets by counting; neighbours come out sorted ascending.
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "lap_host.h"

namespace lap {

static void radix_sort_u64(std::vector<uint64_t> &a, int bits) {
    const int kDigit = 11;
    const size_t n = a.size();
    std::vector<uint64_t> tmp(n);
    std::vector<size_t> cnt(1u << kDigit);
    for (int shift = 0; shift < bits; shift += kDigit) {
        std::fill(cnt.begin(), cnt.end(), 0);
        const uint64_t mask = (1ull << kDigit) - 1;
        for (size_t i = 0; i < n; ++i) ++cnt[(a[i] >> shift) & mask];
        size_t sum = 0;
        for (auto &c : cnt) {
            const size_t t = c;
            c = sum;
            sum += t;
        }
        for (size_t i = 0; i < n; ++i) tmp[cnt[(a[i] >> shift) & mask]++] = a[i];
        a.swap(tmp);
    }
}

static int32_t uf_find(std::vector<int32_t> &par, int32_t x) {
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

int build_host_csr(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst, bool keep_lcc,
                   HostCSR &out, std::string &err) {
    if (n < 1 || n >= (int64_t)1 << 31) {
        err = "n must be in [1, 2^31)";
        return LAP_EINVAL;
    }
    if (n_edges < 0 || (n_edges > 0 && (!src || !dst))) {
        err = "bad edge arrays";
        return LAP_EINVAL;
    }
    std::vector<uint64_t> keys;
    try {
        keys.reserve((size_t)n_edges * 2);
    } catch (...) {
        err = "host allocation failed";
        return LAP_ENOMEM;
    }
    const uint64_t N = (uint64_t)n;
    for (int64_t e = 0; e < n_edges; ++e) {
        const int64_t a = src[e], b = dst[e];
        if (a < 0 || a >= n || b < 0 || b >= n) {
            err = "edge " + std::to_string(e) + " has a node id outside [0, n)";
            return LAP_EINVAL;
        }
        if (a == b) continue;
        keys.push_back((uint64_t)a * N + (uint64_t)b);
        keys.push_back((uint64_t)b * N + (uint64_t)a);
    }
    int bits = 1;
    const uint64_t maxkey = N * N;
    while (bits < 64 && (1ull << bits) < maxkey) ++bits;
    radix_sort_u64(keys, bits);
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());

    // connected components
    std::vector<int32_t> par((size_t)n);
    std::iota(par.begin(), par.end(), 0);
    for (uint64_t k : keys) {
        const int32_t a = (int32_t)(k / N), b = (int32_t)(k % N);
        if (a < b) {
            const int32_t ra = uf_find(par, a), rb = uf_find(par, b);
            if (ra != rb) par[std::max(ra, rb)] = std::min(ra, rb);   // root = smallest id
        }
    }
    std::vector<int64_t> size((size_t)n, 0);
    int64_t ncomp = 0;
    for (int64_t u = 0; u < n; ++u) {
        const int32_t r = uf_find(par, (int32_t)u);
        if (size[r]++ == 0) ++ncomp;
    }
    int32_t keep_root = 0;
    if (ncomp > 1) {
        if (!keep_lcc) {
            err = "graph has " + std::to_string(ncomp) + " connected components";
            return LAP_ENOTCONN;
        }
        // roots are the smallest ids of their components; scanning ids upward
        // and taking the first strict maximum breaks ties by smallest id
        int64_t best = -1;
        for (int64_t u = 0; u < n; ++u)
            if (par[u] == (int32_t)u && size[u] > best) {
                best = size[u];
                keep_root = (int32_t)u;
            }
    }
    std::vector<int32_t> newid((size_t)n, -1);
    out.old_ids.clear();
    for (int64_t u = 0; u < n; ++u)
        if (ncomp == 1 || uf_find(par, (int32_t)u) == keep_root) {
            newid[u] = (int32_t)out.old_ids.size();
            out.old_ids.push_back((int32_t)u);
        }
    const int64_t n2 = (int64_t)out.old_ids.size();
    out.n = n2;
    out.rp.assign((size_t)n2 + 1, 0);
    out.col.clear();
    out.col.reserve(keys.size());
    for (uint64_t k : keys) {
        const int32_t a = newid[k / N], b = newid[k % N];
        if (a < 0 || b < 0) continue;
        ++out.rp[(size_t)a + 1];
        out.col.push_back(b);
    }
    for (int64_t u = 0; u < n2; ++u) out.rp[u + 1] += out.rp[u];
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
