"""The oracle's BFS tree from the landmark (the precomputation of Alg. 1 and
Alg. 3, whose depth is the Delta_G of Thms. 3 and 4), pinned without
reference to itself:
  - every node's depth in the tree equals its hop distance from v, taken from
    scipy's unweighted shortest paths (a library routine);
  - every parent is a graph neighbour one hop closer to v;
  - the parent is the one a breadth-first search with neighbours taken in
    ascending order discovers first.  That rule is rebuilt here level by
    level (each level ordered by its nodes' first-discovering parent, then
    by id) instead of with a queue, so a stack-for-queue or ordering slip in
    the oracle gives different parents."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import graphgen as gg
from oracle import csr, native
from tests.oracle_fixtures import er256, graph


def _cases():
    out = [("er256", er256())]
    s, d = gg.barabasi_albert(2000, 3, 5)
    out.append(("ba2000", csr.build_csr(2000, s, d)))
    s, d = gg.rmat(12, 8, seed=3)
    out.append(("rmat12_lcc", csr.build_csr(1 << 12, s, d, keep_lcc=True)))
    for r, c in ((7, 9), (2, 40), (12, 12)):
        out.append((f"grid{r}x{c}", graph("grid", r, c)))
    out.append(("cycle31", graph("cycle", 31)))
    return out


CASES = _cases()


def _hops(g, v):
    a = sp.csr_matrix((np.ones(len(g.col)), g.col, g.rp), shape=(g.n, g.n))
    return shortest_path(a, unweighted=True, directed=False, indices=[v])[0]


def _level_parents(g, v):
    """Parents of a breadth-first search with ascending neighbour order,
    built one level at a time: the order inside level k+1 is by the
    position of the first level-k node adjacent to it, then by node id."""
    par = np.full(g.n, -1, np.int64)
    seen = np.zeros(g.n, bool)
    seen[v] = True
    level = [v]
    while level:
        pos = {a: i for i, a in enumerate(level)}
        first = {}
        for a in level:
            for b in g.col[g.rp[a]:g.rp[a + 1]]:
                b = int(b)
                if not seen[b] and (b not in first or pos[a] < pos[first[b]]):
                    first[b] = a
        nxt = sorted(first, key=lambda b: (pos[first[b]], b))
        for b in nxt:
            par[b] = first[b]
            seen[b] = True
        level = nxt
    return par


def _roots(g):
    deg = np.diff(g.rp)
    rng = np.random.default_rng(g.n)
    return sorted({int(np.argmax(deg)), 0, g.n - 1, *rng.integers(0, g.n, 3).tolist()})


@pytest.mark.parametrize("name,g", CASES, ids=[c[0] for c in CASES])
def test_bfs_tree_depth_is_hop_distance(name, g):
    for v in _roots(g):
        par = native.bfs_tree(g, v)
        hops = _hops(g, v)
        assert np.all(np.isfinite(hops)), "fixtures are connected"
        assert par[v] == -1
        depth = np.full(g.n, -1, np.int64)
        depth[v] = 0
        # depth by climbing the parent pointers (each climb is bounded by n)
        for u in range(g.n):
            path, x = [], u
            while depth[x] < 0:
                path.append(x)
                x = int(par[x])
                assert x >= 0 and len(path) <= g.n, f"node {u}: parent chain leaves the tree"
            for i, y in enumerate(reversed(path)):
                depth[y] = depth[x] + i + 1
        np.testing.assert_array_equal(depth, hops.astype(np.int64))
        for u in range(g.n):
            if u == v:
                continue
            p = int(par[u])
            row = g.col[g.rp[u]:g.rp[u + 1]]
            assert p in row, f"root {v}: parent {p} of {u} is not a neighbour"
            assert hops[p] == hops[u] - 1


@pytest.mark.parametrize("name,g", CASES, ids=[c[0] for c in CASES])
def test_bfs_tree_parent_is_first_discovered(name, g):
    for v in _roots(g):
        np.testing.assert_array_equal(native.bfs_tree(g, v).astype(np.int64), _level_parents(g, v))


def test_level_rule_tells_queue_from_stack():
    """The level-by-level rule is sharp enough to catch a depth-first slip:
    on a 4x4 grid from a corner a stack order gives a different tree."""
    g = graph("grid", 4, 4)
    v = 0
    par_dfs = np.full(g.n, -1, np.int64)
    seen = np.zeros(g.n, bool)
    seen[v] = True
    stack = [v]
    while stack:
        a = stack.pop()
        for b in g.col[g.rp[a]:g.rp[a + 1]]:
            b = int(b)
            if not seen[b]:
                seen[b] = True
                par_dfs[b] = a
                stack.append(b)
    assert not np.array_equal(par_dfs, _level_parents(g, v))
