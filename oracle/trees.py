"""Brute-force spanning trees of tiny graphs (test infrastructure only).

Enumerates every (n-1)-edge subset and keeps the acyclic ones; each tree is
returned as the parent array obtained by orienting it toward the root v
(parent[v] = -1), the same form as Wilson's next[] array (Sec. 3.4).  The
count equals det(L_v) by the matrix-tree theorem.
"""
from __future__ import annotations

import itertools

import numpy as np


def undirected_edges(g):
    out = []
    for u in range(g.n):
        for w in g.col[g.rp[u]:g.rp[u + 1]]:
            if u < w:
                out.append((u, int(w)))
    return out


def spanning_trees(g, root):
    edges = undirected_edges(g)
    n = g.n
    trees = []
    for sub in itertools.combinations(range(len(edges)), n - 1):
        par = list(range(n))

        def find(x):
            while par[x] != x:
                par[x] = par[par[x]]
                x = par[x]
            return x

        ok = True
        for e in sub:
            a, b = find(edges[e][0]), find(edges[e][1])
            if a == b:
                ok = False
                break
            par[a] = b
        if not ok:
            continue
        adj = [[] for _ in range(n)]
        for e in sub:
            a, b = edges[e]
            adj[a].append(b)
            adj[b].append(a)
        parent = np.full(n, -1, np.int32)
        seen = [False] * n
        seen[root] = True
        stack = [root]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if not seen[y]:
                    seen[y] = True
                    parent[y] = x
                    stack.append(y)
        trees.append(tuple(parent.tolist()))
    return trees
