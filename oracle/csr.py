"""Oracle graph preparation (test infrastructure only).

The paper works on a simple, undirected, connected graph (Sec. 2) and uses
the highest-degree node as the landmark v (Sec. 6.1).  From a raw edge list
this module builds that graph in CSR form with plain numpy/scipy steps:
  1. treat every pair as an undirected edge: add both orientations;
  2. drop self-loops and merge duplicate pairs;
  3. optionally keep only the largest connected component (ties: the
     component holding the smallest node id) and renumber its nodes by
     ascending original id; otherwise a disconnected graph is an error;
  4. optionally (degree_order) number the nodes by decreasing degree, ties
     by increasing id after step 3 -- a relabelling of the same graph;
  5. rows list neighbours in ascending order.
Landmark: the node of maximum degree, lowest id on ties.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclass
class Graph:
    n: int
    rp: np.ndarray          # int64 [n+1]
    col: np.ndarray         # int32 [nnz], nnz = 2m
    old_ids: np.ndarray     # int32 [n]: original id of each node

    @property
    def nnz(self):
        return int(self.rp[-1])

    @property
    def deg(self):
        return np.diff(self.rp)


class NotConnected(ValueError):
    pass


def build_csr(n, src, dst, keep_lcc=False, degree_order=False) -> Graph:
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    if len(src) and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("node id out of range")
    u = np.concatenate([src, dst])
    v = np.concatenate([dst, src])
    keep = u != v
    key = np.unique(u[keep] * n + v[keep])           # sorted by (row, col), duplicates merged
    u = key // n
    v = key % n
    old_ids = np.arange(n, dtype=np.int64)
    A = sp.csr_matrix((np.ones(len(u), np.int8), (u, v)), shape=(n, n))
    ncomp, lab = connected_components(A, directed=False)
    if ncomp > 1:
        if not keep_lcc:
            raise NotConnected(f"graph has {ncomp} connected components")
        sizes = np.bincount(lab, minlength=ncomp)
        best = sizes.max()
        # component with the largest size; ties -> the one containing the smallest id
        first_id = np.full(ncomp, n, np.int64)
        np.minimum.at(first_id, lab, np.arange(n))
        cands = np.nonzero(sizes == best)[0]
        c = cands[np.argmin(first_id[cands])]
        old_ids = np.nonzero(lab == c)[0]
        newid = np.full(n, -1, np.int64)
        newid[old_ids] = np.arange(len(old_ids))
        m = (newid[u] >= 0) & (newid[v] >= 0)
        u, v = newid[u[m]], newid[v[m]]
        n = len(old_ids)
    if degree_order:
        deg = np.bincount(u, minlength=n)
        order = np.lexsort((np.arange(n), -deg))     # by degree descending, then id
        rank = np.empty(n, np.int64)
        rank[order] = np.arange(n)
        u, v = rank[u], rank[v]
        key = np.sort(u * n + v)                       # rows ascending again
        u, v = key // n, key % n
        old_ids = old_ids[order]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, u + 1, 1)
    rp = np.cumsum(rp)
    return Graph(n=int(n), rp=rp, col=v.astype(np.int32), old_ids=old_ids.astype(np.int32))


def landmark(g: Graph) -> int:
    """Highest-degree node, lowest id on ties."""
    return int(np.argmax(g.deg))
