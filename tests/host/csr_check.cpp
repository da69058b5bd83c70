// Host-only check of the threaded CSR builder (build_host_csr), built by
// tests/test_host_sanitizers.py under AddressSanitizer + UBSan and under
// ThreadSanitizer.  Random multigraphs with self-loops, duplicate edges and
// several components are built with and without keeping the largest
// component, and compared with a plain sort-and-unique construction; the
// degree-ordered numbering is compared with the plain one.  Two
// graphs are large enough (over 2^20 row entries) for every threaded pass.
#include <algorithm>
#include <cstdio>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "lap_host.h"

using namespace lap;

namespace {

int32_t find(std::vector<int32_t> &p, int32_t x) {
    while (p[x] != x) x = p[x] = p[p[x]];
    return x;
}

// returns the number of mismatches for one graph and one flag setting
int check(int64_t n, const std::vector<int32_t> &s, const std::vector<int32_t> &d, bool keep) {
    HostCSR g;
    std::string err;
    const int rc = build_host_csr(n, (int64_t)s.size(), s.data(), d.data(), keep, g, err);
    std::vector<std::pair<int32_t, int32_t>> arcs;
    std::vector<int32_t> par(n);
    std::iota(par.begin(), par.end(), 0);
    for (size_t i = 0; i < s.size(); ++i) {
        if (s[i] == d[i]) continue;
        arcs.emplace_back(s[i], d[i]);
        arcs.emplace_back(d[i], s[i]);
        par[find(par, s[i])] = find(par, d[i]);
    }
    std::sort(arcs.begin(), arcs.end());
    arcs.erase(std::unique(arcs.begin(), arcs.end()), arcs.end());
    std::vector<int64_t> size(n, 0);
    int64_t comps = 0;
    for (int64_t u = 0; u < n; ++u) comps += find(par, (int32_t)u) == u, ++size[find(par, (int32_t)u)];
    if (!keep && comps > 1) return rc == LAP_ENOTCONN ? 0 : 1;
    if (rc != LAP_OK) {
        std::printf("n=%ld keep=%d: rc %d (%s)\n", (long)n, (int)keep, rc, err.c_str());
        return 1;
    }
    // the kept nodes: all of them, or the largest component (its size is unique
    // to check; which of several equal-size components is kept is not checked)
    const int64_t big = *std::max_element(size.begin(), size.end());
    if (g.n != (keep ? big : n) || (int64_t)g.rp.size() != g.n + 1) {
        std::printf("n=%ld keep=%d: %ld nodes kept\n", (long)n, (int)keep, (long)g.n);
        return 1;
    }
    std::vector<int32_t> to_new(n, -1);
    for (int64_t u = 0; u < g.n; ++u) {
        const int32_t old = keep ? g.old_ids[u] : (int32_t)u;
        if (old < 0 || old >= n || (u > 0 && keep && g.old_ids[u - 1] >= old)) return 1;   // ascending old ids
        to_new[old] = (int32_t)u;
    }
    std::vector<std::vector<int32_t>> want(g.n);
    for (auto &a : arcs)
        if (to_new[a.first] >= 0) want[to_new[a.first]].push_back(to_new[a.second]);
    int bad = 0;
    for (int64_t u = 0; u < g.n; ++u) {
        std::sort(want[u].begin(), want[u].end());
        if (!std::equal(want[u].begin(), want[u].end(), g.col.begin() + g.rp[u], g.col.begin() + g.rp[u + 1]) ||
            (int64_t)want[u].size() != g.rp[u + 1] - g.rp[u])
            ++bad;
    }
    if (bad) std::printf("n=%ld keep=%d: %d rows differ\n", (long)n, (int)keep, bad);
    return bad;
}

// the same graph numbered by decreasing degree (ties by increasing original
// id): the same kept nodes, the same edges, rows ascending
int check_degree_order(int64_t n, const std::vector<int32_t> &s, const std::vector<int32_t> &d, bool keep) {
    HostCSR a, b;
    std::string err;
    const int ra = build_host_csr(n, (int64_t)s.size(), s.data(), d.data(), keep, a, err);
    const int rb = build_host_csr(n, (int64_t)s.size(), s.data(), d.data(), keep, b, err, true);
    if (ra != rb) return 1;
    if (ra != LAP_OK) return 0;
    if (a.n != b.n || a.rp[a.n] != b.rp[b.n]) return 1;
    const int64_t m = a.n;
    // original id of every node of a
    std::vector<int32_t> orig_a(m), orig_b(m);
    for (int64_t u = 0; u < m; ++u) {
        orig_a[u] = keep ? a.old_ids[u] : (int32_t)u;
        orig_b[u] = b.old_ids[u];
    }
    std::vector<int32_t> sa = orig_a, sb = orig_b;
    std::sort(sa.begin(), sa.end());
    std::sort(sb.begin(), sb.end());
    if (sa != sb) return 1;
    std::vector<int32_t> a_of_orig(n, -1);
    for (int64_t u = 0; u < m; ++u) a_of_orig[orig_a[u]] = (int32_t)u;
    int bad = 0;
    for (int64_t v = 0; v < m; ++v) {
        const int64_t dv = b.rp[v + 1] - b.rp[v];
        if (v > 0) {
            const int64_t dp = b.rp[v] - b.rp[v - 1];
            if (dp < dv || (dp == dv && orig_b[v - 1] >= orig_b[v])) ++bad;
        }
        const int32_t u = a_of_orig[orig_b[v]];
        if (u < 0 || a.rp[u + 1] - a.rp[u] != dv) {
            ++bad;
            continue;
        }
        std::vector<int32_t> ra_row, rb_row;
        for (int64_t j = a.rp[u]; j < a.rp[u + 1]; ++j) ra_row.push_back(orig_a[a.col[j]]);
        for (int64_t j = b.rp[v]; j < b.rp[v + 1]; ++j) {
            if (j > b.rp[v] && b.col[j - 1] >= b.col[j]) ++bad;
            rb_row.push_back(orig_b[b.col[j]]);
        }
        std::sort(ra_row.begin(), ra_row.end());
        std::sort(rb_row.begin(), rb_row.end());
        if (ra_row != rb_row) ++bad;
    }
    if (bad) std::printf("n=%ld keep=%d degree order: %d mismatches\n", (long)n, (int)keep, bad);
    return bad;
}

}  // namespace

int main() {
    std::mt19937_64 rng(7);
    int bad = 0;
    for (int it = 0; it < 62; ++it) {
        const bool large = it >= 60;
        const int64_t n = large ? 300000 : 1 + (int64_t)(rng() % 2000);
        const int64_t m = large ? 700000 : (int64_t)(rng() % (3 * n + 1));
        std::vector<int32_t> s((size_t)m), d((size_t)m);
        for (int64_t i = 0; i < m; ++i) {
            s[i] = (int32_t)(rng() % n);
            d[i] = (rng() % 7 == 0) ? s[i] : (int32_t)(rng() % n);
            if (rng() % 5 == 0 && i > 0) { s[i] = s[i - 1]; d[i] = d[i - 1]; }   // duplicates
        }
        bad += check(n, s, d, false);
        bad += check(n, s, d, true);
        bad += check_degree_order(n, s, d, true);
        if (it % 4 == 0) bad += check_degree_order(n, s, d, false);
    }
    HostCSR g;
    std::string err;
    bad += build_host_csr(0, 0, nullptr, nullptr, true, g, err) != LAP_EINVAL;
    std::printf("%s (%d mismatches)\n", bad ? "FAIL" : "ok", bad);
    return bad != 0;
}
