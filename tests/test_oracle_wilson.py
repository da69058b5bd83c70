"""Pins for the oracle's Wilson sampler and loop-included paths: the
stack-representation worked example (Fig. 1), order independence of the
stack view, uniformity over all spanning trees (brute force), and the
exact expectations of the counts (Lemma 4; total = Tr (I-P_v)^{-1})."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import csr, dense, native, trees
from tests.oracle_fixtures import er256, graph, ints, read_golden


def _fig1():
    stacks, orders, nxt, paths = {}, [], None, []
    for tag, rest in read_golden("fig1_stacks.txt"):
        if tag == "stack":
            v = ints(rest)
            stacks[v[0]] = v[1:]
        elif tag == "order":
            a, b = rest.split(";")
            orders.append((ints(a), ints(b)))
        elif tag == "next":
            nxt = ints(rest)
        elif tag == "path":
            a, b = rest.split(";")
            paths.append((int(a), ints(b)))
    return stacks, orders, nxt, paths


def test_fig1_trajectories_tree_and_draws():
    stacks, orders, nxt, _ = _fig1()
    for order, traj in orders:
        r = native.wilson_scripted(4, 3, stacks, order)
        assert r["trace"].tolist() == traj
        assert r["next"].tolist() == nxt
        assert r["draws"].tolist() == [2, 2, 1, 0]
        assert r["total"] == 5


def test_fig1_loop_included_paths():
    stacks, _, _, paths = _fig1()
    for s, p in paths:
        assert native.loop_included_path(4, 3, s, stacks=stacks).tolist() == p


def test_scripted_stack_exhaustion_is_an_error():
    with pytest.raises(ValueError):
        native.wilson_scripted(4, 3, {0: [1], 1: [0], 2: [3]}, [0, 1, 2])


@settings(max_examples=40, deadline=None)
@given(seed=st.integers(0, 2**32), sample=st.integers(0, 1000), perm_seed=st.integers(0, 2**32))
def test_order_independence(seed, sample, perm_seed):
    g = graph("grid", 3, 4)
    root = 5
    rng = np.random.default_rng(perm_seed)
    base = native.wilson_ordered(g, root, sample, seed,
                                 [u for u in range(g.n) if u != root])
    order = rng.permutation([u for u in range(g.n) if u != root])
    other = native.wilson_ordered(g, root, sample, seed, order)
    assert base["draws"].tolist() == other["draws"].tolist()
    assert base["next"].tolist() == other["next"].tolist()
    assert base["total"] == other["total"] == int(base["draws"].sum())


def test_next_is_a_spanning_tree_toward_root():
    g = er256()
    v = csr.landmark(g)
    r = native.wilson(g, v, 8, 1, keep=range(8))
    for q in range(8):
        nxt = r["next"][q]
        assert nxt[v] == -1
        for u in range(g.n):
            if u == v:
                continue
            assert nxt[u] in g.col[g.rp[u]:g.rp[u + 1]]     # a tree edge is a graph edge
            x, steps = u, 0
            while x != v:
                x = nxt[x]
                steps += 1
                assert steps <= g.n
        assert r["y1"][q] == r["draws"][q].sum()
        assert (r["draws"][q][np.arange(g.n) != v] >= 1).all()


@pytest.mark.parametrize("name,args,root", [("diamond", (), 3), ("grid", (2, 3), 0),
                                            ("cycle", (5,), 2), ("complete", (4,), 1)])
def test_wilson_uniform_over_spanning_trees(name, args, root):
    g = graph(name, *args)
    all_trees = trees.spanning_trees(g, root)
    L = dense.laplacian(g)
    keep = [i for i in range(g.n) if i != root]
    assert len(all_trees) == round(np.linalg.det(L[np.ix_(keep, keep)]))   # matrix-tree theorem
    omega = 200 * len(all_trees)
    r = native.wilson(g, root, omega, 11, keep=range(omega), want_y1=False)
    idx = {t: i for i, t in enumerate(all_trees)}
    counts = np.zeros(len(all_trees))
    for q in range(omega):
        counts[idx[tuple(r["next"][q].tolist())]] += 1
    exp = omega / len(all_trees)
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    dof = len(all_trees) - 1
    # 6-sigma bound of the chi-square distribution
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_draw_count_expectations_er256():
    g = er256()
    v = csr.landmark(g)
    omega = 4096
    r = native.wilson(g, v, omega, 1)
    e = dense.expected_counts(g, v)
    # total draws per sample: mean Tr N (Sec. 5, LEWalk-KC y1)
    y1 = r["y1"].astype(float)
    z = (y1.mean() - e["total"]) / (y1.std(ddof=1) / math.sqrt(omega))
    assert abs(z) < 4.0
    # per-node draws: E = N_uu (Lemma 4); per-sample counts are independent
    # across samples, so each node's mean is a z-test; require the max over
    # nodes within a Bonferroni bound and the bulk within 3 sigma
    samples = native.wilson(g, v, omega, 1, keep=range(omega), want_y1=False)["draws"]
    mean = samples.mean(0)
    sd = samples.std(0, ddof=1) / math.sqrt(omega)
    mask = np.arange(g.n) != v
    zz = (mean[mask] - e["draws"][mask]) / sd[mask]
    assert np.abs(zz).max() < 4.6
    assert (np.abs(zz) < 3).mean() > 0.98
    assert (r["Y1"].sum(0) == samples.sum(0)).all()


def test_block_split_and_sample_ranges_are_consistent():
    g = graph("grid", 3, 3)
    full = native.wilson(g, 4, 100, 5, B=7)
    parts = [native.wilson(g, 4, 100, 5, sample_begin=a, n_samples=b - a, B=7)
             for a, b in [(0, 13), (13, 64), (64, 100)]]
    assert (sum(p["Y1"] for p in parts) == full["Y1"]).all()
    assert np.concatenate([p["y1"] for p in parts]).tolist() == full["y1"].tolist()
    # sample i lands in block floor(i*B/omega)
    one = [native.wilson(g, 4, 100, 5, sample_begin=i, n_samples=1, B=7)["Y1"] for i in (0, 14, 15, 99)]
    assert one[0][0].sum() > 0 and one[1][0].sum() > 0 and one[2][1].sum() > 0 and one[3][6].sum() > 0


def test_threads_do_not_change_counts():
    g = er256()
    v = csr.landmark(g)
    a = native.wilson(g, v, 300, 3, B=4, threads=1)
    b = native.wilson(g, v, 300, 3, B=4, threads=4)
    assert (a["Y1"] == b["Y1"]).all() and (a["y1"] == b["y1"]).all()
