"""Pins for the oracle's graph preparation against networkx (a library
routine) and hand-checked cases."""
import networkx as nx
import numpy as np
import pytest

import graphgen as gg
from oracle import csr


def _nx_reference(n, src, dst, keep_lcc):
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(src, dst) if a != b)
    if keep_lcc:
        comps = sorted(nx.connected_components(G), key=lambda c: (-len(c), min(c)))
        nodes = sorted(comps[0])
    else:
        nodes = list(range(n))
    idx = {u: i for i, u in enumerate(nodes)}
    rows = [sorted(idx[w] for w in G.neighbors(u) if w in idx) for u in nodes]
    return nodes, rows


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_networkx_with_lcc(seed):
    src, dst = gg.rmat(8, 4, seed=seed)
    g = csr.build_csr(256, src, dst, keep_lcc=True)
    nodes, rows = _nx_reference(256, src, dst, True)
    assert g.old_ids.tolist() == nodes
    for u in range(g.n):
        assert g.col[g.rp[u]:g.rp[u + 1]].tolist() == rows[u]


def test_duplicates_self_loops_and_orientation():
    g = csr.build_csr(3, [0, 1, 1, 2, 2], [1, 0, 1, 1, 0])
    assert g.rp.tolist() == [0, 2, 4, 6]
    assert g.col.tolist() == [1, 2, 0, 2, 0, 1]


def test_disconnected_without_lcc_raises():
    with pytest.raises(csr.NotConnected):
        csr.build_csr(4, [0, 2], [1, 3])


def test_lcc_tie_goes_to_smallest_id():
    g = csr.build_csr(5, [3, 0], [4, 1], keep_lcc=True)
    assert g.old_ids.tolist() == [0, 1]


def test_landmark_lowest_id_on_ties():
    g = csr.build_csr(4, [0, 1, 2, 3], [1, 2, 3, 0])
    assert csr.landmark(g) == 0


@pytest.mark.parametrize("seed,keep", [(0, True), (1, True), (5, False)])
def test_degree_order_is_a_relabelling(seed, keep):
    """degree_order numbers the nodes by decreasing degree, ties by increasing
    id, and is otherwise the same graph: networkx's edge set (in original
    ids) and degrees are unchanged, rows stay ascending."""
    if keep:
        src, dst = gg.rmat(9, 6, seed=seed)
        n = 512
    else:
        src, dst = gg.barabasi_albert(600, 3, seed)
        n = 600
    g = csr.build_csr(n, src, dst, keep_lcc=keep, degree_order=True)
    nodes, rows = _nx_reference(n, src, dst, keep)
    G = nx.Graph()
    G.add_edges_from((int(a), int(b)) for a, b in zip(src, dst) if a != b)
    assert sorted(g.old_ids.tolist()) == nodes
    deg = np.diff(g.rp)
    assert np.all(deg[:-1] >= deg[1:])
    ties = deg[:-1] == deg[1:]
    assert np.all(g.old_ids[:-1][ties] < g.old_ids[1:][ties])
    for u in range(g.n):
        row = g.col[g.rp[u]:g.rp[u + 1]]
        assert np.all(np.diff(row) > 0)
        assert sorted(g.old_ids[row].tolist()) == sorted(G.neighbors(int(g.old_ids[u])))
    assert csr.landmark(g) == 0


def test_degree_order_hand_case():
    # a path 0-1-2 plus 2-3 and 2-4: node 2 (degree 3) first, then node 1
    # (degree 2), then 0, 3, 4 (degree 1, by id)
    g = csr.build_csr(5, [0, 1, 2, 2], [1, 2, 3, 4], degree_order=True)
    assert g.old_ids.tolist() == [2, 1, 0, 3, 4]
    assert g.rp.tolist() == [0, 3, 5, 6, 7, 8]
    assert g.col.tolist() == [1, 3, 4, 0, 2, 1, 0, 0]
