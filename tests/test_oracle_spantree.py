"""The SpanTree estimators' oracle (Alg. 1 for closeness, Alg. 3 for Kemeny's
constant), pinned without reference to itself:
  - averaged over every spanning tree of small graphs (each tree equally
    likely, as Wilson samples them), the per-tree sums equal the dense
    quantities exactly: x1(u) -> (L_v^{-1})_uu, x2(u)/n -> (1/n)(L_v^{-1} 1)_u,
    sum_u d_u x1(u) -> Tr((I - P_v)^{-1}), sum_u d_u x2(u)/2m ->
    d^T L_v^{-1} d / 2m (Sec. 4.1, Sec. 5.2);
  - the tree-averaged edge currents of Fig. 3 (golden values);
  - path support equals subtree sums found by brute force, and the DFS
    intervals nest exactly along tree ancestry;
  - the sampled estimator over Wilson trees is within its standard error of
    the dense pseudo-inverse and of Kemeny's constant on the small ER graph."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr, dense, estimators, native, trees
from tests.oracle_fixtures import er256, graph, read_golden


def _tiny():
    out = [graph("diamond"), graph("fig1_graph"), graph("grid", 3, 3), graph("cycle", 7), graph("star", 6),
           graph("path", 5), graph("complete", 5)]
    s = np.array([0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 5, 6, 7])
    d = np.array([1, 2, 3, 4, 5, 4, 6, 5, 7, 8, 8, 7, 8])
    out.append(csr.build_csr(9, s, d))
    return out


def _averages(g, v):
    T = trees.spanning_trees(g, v)
    par = native.bfs_tree(g, v)
    deg = g.deg.astype(np.int64)
    a1 = np.zeros(g.n)
    a2 = np.zeros(g.n)
    k1 = k2 = 0.0
    for t in T:
        r = native.spantree_tree(g, v, t, bfs_par=par)
        a1 += r["x1"]
        a2 += r["x2"]
        rk = native.spantree_tree(g, v, t, weights=deg, bfs_par=par)
        k1 += float(deg @ rk["x1"])
        k2 += float(deg @ rk["x2"])
    m = len(T)
    return a1 / m, a2 / m, k1 / m, k2 / m


@pytest.mark.parametrize("gi", range(8))
def test_tree_averages_equal_dense_quantities(gi):
    g = _tiny()[gi]
    L = dense.laplacian(g)
    d = np.diag(L)
    for v in range(g.n):
        Lvi = dense.lv_inv(L, v)
        a1, a2, k1, k2 = _averages(g, v)
        np.testing.assert_allclose(a1, np.diag(Lvi), atol=1e-12)
        np.testing.assert_allclose(a2, Lvi.sum(1), atol=1e-12)
        assert k1 == pytest.approx(np.trace(dense.walk_green(L, v)), abs=1e-9)
        dv = d.copy()
        dv[v] = 0
        assert k2 / d.sum() == pytest.approx(dv @ Lvi @ dv / d.sum(), abs=1e-12)
        # assembled as in Alg. 1 and Alg. 3 from exact averages
        est = a1 - 2 * a2 / g.n + a2.sum() / g.n ** 2
        np.testing.assert_allclose(est, np.diag(dense.pinv_eigh(L)), atol=1e-12)
        assert k1 - k2 / d.sum() == pytest.approx(dense.kemeny_spectral(g), abs=1e-9)


def test_fig3_currents_are_tree_averages():
    g = graph("diamond")
    v = 2
    flows = {(int(a), int(b)): float(x) for a, b, x in
             (r.split() for t, r in read_golden("diamond.txt") if t == "fig3_flow")}
    T = trees.spanning_trees(g, v)
    par = native.bfs_tree(g, v)
    got = {e: 0.0 for e in flows}
    for t in T:
        ps = native.spantree_tree(g, v, t, bfs_par=par)["ps"] / g.n
        for (a, b) in flows:
            got[(a, b)] += (ps[a] if t[a] == b else 0.0) - (ps[b] if t[b] == a else 0.0)
    for e, x in flows.items():
        assert got[e] / len(T) == pytest.approx(x, abs=1e-12), e


def test_path_support_and_dfs_intervals_by_brute_force():
    g = er256()
    v = csr.landmark(g)
    w = native.wilson(g, v, 3, 5, keep=[0, 1, 2])
    deg = g.deg.astype(np.int64)
    for q in range(3):
        t = w["next"][q]
        anc = []       # ancestors-or-self of every node, walking the tree
        for u in range(g.n):
            a, chain = u, []
            while a != v:
                chain.append(a)
                a = t[a]
            anc.append(chain)
        r = native.spantree_tree(g, v, t, weights=deg)
        ps = np.zeros(g.n, np.int64)
        for u in range(g.n):
            for a in anc[u]:
                ps[a] += deg[u]
        assert np.array_equal(r["ps"], ps)
        vis, fin = r["vis"], r["fin"]
        for u in range(g.n):
            inside = {a for a in range(g.n) if vis[a] <= vis[u] and fin[u] <= fin[a]}
            assert inside == set(anc[u]) | {v}


def test_sampler_uses_the_wilson_trees():
    g = er256()
    v = csr.landmark(g)
    w = native.wilson(g, v, 40, 9, keep=list(range(40)))
    r = native.spantree(g, v, 40, 9, 1)
    par = native.bfs_tree(g, v)
    X1 = np.zeros(g.n, np.int64)
    X2 = np.zeros(g.n, np.int64)
    for q in range(40):
        t = native.spantree_tree(g, v, w["next"][q], bfs_par=par)
        X1 += t["x1"]
        X2 += t["x2"]
    assert np.array_equal(r["X1"], X1) and np.array_equal(r["X2"], X2)
    k = native.spantree(g, v, 40, 9, 2)
    deg = g.deg.astype(np.int64)
    for q in (0, 17, 39):
        t = native.spantree_tree(g, v, w["next"][q], weights=deg, bfs_par=par)
        assert k["s1"][q] == deg @ t["x1"] and k["s2"][q] == deg @ t["x2"]


def test_sampled_estimates_within_standard_errors():
    g = er256()
    v = csr.landmark(g)
    L = dense.laplacian(g)
    Ld = dense.pinv_eigh(L)
    omega, B = 4096, 32
    blocks = []
    for b in range(B):
        r = native.spantree(g, v, omega // B, 1, 1, sample_begin=b * (omega // B))
        blocks.append(estimators.spantree_diag(r["X1"], r["X2"], omega // B, g.n))
    blocks = np.array(blocks)
    est = blocks.mean(0)
    se = blocks.std(0, ddof=1) / np.sqrt(B)
    z = (est - np.diag(Ld)) / se
    assert np.max(np.abs(z)) < 4.6 and np.mean(np.abs(z) < 3) >= 0.97
    k = native.spantree(g, v, omega, 1, 2)
    kap, kse = estimators.spantree_kemeny(k["s1"], k["s2"], int(g.deg.sum()))
    assert abs(kap - dense.kemeny_spectral(g)) < 3 * kse
