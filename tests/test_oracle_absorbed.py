"""Pins for the oracle's v-absorbed walks: start distributions (uniform over
all of V for the closeness estimator, stationary for Kemeny), visit-count
expectations (Lemmas 1 and 5), walk-length expectations, loop-included paths
having the absorbed-walk distribution (Lemma 4), and exact small cases."""
import math

import numpy as np
import pytest

from oracle import csr, dense, native
from tests.oracle_fixtures import er256, graph


def test_star_walks_are_one_step():
    g = graph("star", 7)
    r = native.absorbed(g, 0, 2000, 4, 1, want_start=True)
    st = r["start"]
    assert set(np.unique(st)) <= set(range(7))
    assert (r["len"] == (st != 0)).all()              # a leaf needs one move, the root none
    assert (r["Y2"][0][0] == 0) and r["Y2"][0][1:].sum() == (st != 0).sum()


def test_uniform_start_distribution():
    g = graph("cycle", 10)
    r = native.absorbed(g, 3, 50_000, 9, 1, want_start=True, want_y2=False)
    cnt = np.bincount(r["start"], minlength=10)
    exp = 5000.0
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < 9 + 6 * math.sqrt(18)
    assert cnt[3] > 0                                  # the root itself is a possible start


def test_stationary_start_distribution():
    g = graph("barabasi_albert", 30, 2, 5)
    r = native.absorbed(g, 0, 60_000, 9, 2, want_start=True, want_y2=False)
    cnt = np.bincount(r["start"], minlength=g.n)
    exp = 60_000 * g.deg / g.nnz
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < (g.n - 1) + 6 * math.sqrt(2 * (g.n - 1))


def test_visit_and_length_expectations_er256():
    g = er256()
    v = csr.landmark(g)
    e = dense.expected_counts(g, v)
    W = 8192
    for tag, key in ((1, "len_uniform"), (2, "len_stationary")):
        r = native.absorbed(g, v, W, 1, tag)
        ln = r["len"].astype(float)
        z = (ln.mean() - e[key]) / (ln.std(ddof=1) / math.sqrt(W))
        assert abs(z) < 4.0
        assert r["Y2"].sum() == r["len"].sum()        # every move departs from a node != v
    r = native.absorbed(g, v, W, 2, 1, B=32)
    est = r["Y2"].astype(float)                       # [B, n] block counts
    mean = est.sum(0) / W
    se = est.std(0, ddof=1) * math.sqrt(32) / W      # batch means
    mask = np.arange(g.n) != v
    zz = (mean[mask] - e["visits_uniform"][mask]) / se[mask]
    assert np.abs(zz).max() < 5.0
    assert (np.abs(zz) < 3).mean() > 0.97


def test_trace_is_a_walk_to_root():
    g = graph("grid", 4, 4)
    r = native.absorbed(g, 5, 40, 3, 1, trace_walk=17, trace_cap=10_000)
    tr = r["trace"]
    assert tr[-1] == 5 and (tr[:-1] != 5).all()
    assert len(tr) - 1 == r["len"][17]
    for a, b in zip(tr[:-1], tr[1:]):
        assert b in g.col[g.rp[a]:g.rp[a + 1]]


def test_loop_included_path_has_absorbed_walk_law():
    # Lemma 4: P[s] read from the stacks of a Wilson sample is distributed as a
    # v-absorbed walk from s; compare mean lengths with h(s, v)
    g = graph("grid", 3, 3)
    v, s = 0, 8
    L = dense.laplacian(g)
    h = dense.walk_green(L, v)[s].sum()
    lens = [len(native.loop_included_path(g.n, v, s, g=g, sample=i, seed=21)) - 1 for i in range(6000)]
    lens = np.asarray(lens, float)
    z = (lens.mean() - h) / (lens.std(ddof=1) / math.sqrt(len(lens)))
    assert abs(z) < 4.0


def test_loop_included_path_only_uses_drawn_entries():
    # every departure of P[s] from u reads an entry of S[u] that the Wilson
    # sample also drew, so counts along the path never exceed draws[u]
    g = er256()
    v = csr.landmark(g)
    r = native.wilson(g, v, 3, 8, keep=[0, 1, 2], want_y1=False)
    for q in range(3):
        for s in (0, 100, 200):
            if s == v:
                continue
            p = native.loop_included_path(g.n, v, s, g=g, sample=q, seed=8)
            uses = np.bincount(p[:-1], minlength=g.n)
            assert (uses <= r["draws"][q]).all()


def test_single_node_graph_walks_are_empty():
    """One node, no edges: both kinds of walk start at v and have length 0,
    so Kemeny's constant of a single node is 0 (Sec. 2, empty spectrum sum)."""
    g = csr.build_csr(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    for tag in (1, 2):
        a = native.absorbed(g, 0, 16, 1, tag)
        assert (a["len"] == 0).all() and (a["Y2"] == 0).all()


def test_loop_included_paths_driver():
    """Loop-included paths of Wilson samples (Sec. 3.4), started where the
    absorbed walks of the same index start:
      - each path is the one the single-path routine reads from the stacks;
      - a path never uses more entries of a stack than the sample drew there
        (every entry it uses is popped by Wilson's run, or is the top);
      - departures and lengths have the absorbed walks' expectations."""
    g = er256()
    v = csr.landmark(g)
    r = native.loop_included(g, v, 30, 5, 1)
    starts = native.absorbed(g, v, 30, 5, 1, want_y2=False, want_start=True)["start"]
    w = native.wilson(g, v, 30, 5, keep=list(range(30)), want_y1=False)
    for i in range(30):
        tr = native.loop_included_path(g.n, v, int(starts[i]), g=g, sample=i, seed=5)
        assert len(tr) - 1 == r["len"][i]
        used = np.bincount(tr[:-1], minlength=g.n)
        assert (used <= w["draws"][i]).all()
    L = dense.laplacian(g)
    Lvi = dense.lv_inv(L, v)
    d = np.diag(L)
    omega = 20000
    u = native.loop_included(g, v, omega, 1, 1, B=50)
    ln = u["len"].astype(float)
    exact = (Lvi @ d).sum() / g.n
    assert abs(ln.mean() - exact) < 3.5 * ln.std(ddof=1) / math.sqrt(omega)
    blocks = u["Y2"] / (omega / 50)
    want = d / g.n * Lvi.sum(1)
    z = (blocks.mean(0) - want) / (blocks.std(0, ddof=1) / math.sqrt(50))
    z = z[np.arange(g.n) != v]
    assert np.max(np.abs(z)) < 4.8 and np.mean(np.abs(z) < 3) >= 0.97
    p = native.loop_included(g, v, omega, 2, 2, want_y2=False)
    lp = p["len"].astype(float)
    dv = d.copy()
    dv[v] = 0
    assert abs(lp.mean() - dv @ Lvi @ dv / d.sum()) < 3.5 * lp.std(ddof=1) / math.sqrt(omega)
