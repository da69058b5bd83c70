"""Pins for the oracle's query walks and query assembly: expectations of the
per-walk counts against (L_v^{-1}) from a dense solve (Lemma 1; the
normalised-length lemma of Sec. 4.3), the assembled closeness and
resistance against the dense pseudo-inverse, and exactness when the
expectations themselves are plugged in."""
import math

import numpy as np
import pytest

from oracle import csr, dense, estimators, native
from tests.oracle_fixtures import er256, graph


def test_walk_count_expectations():
    g = graph("grid", 4, 4)
    v = 0
    L = dense.laplacian(g)
    Lvi = dense.lv_inv(L, v)
    d = g.deg
    for s, t in ((15, 6), (5, 10)):
        W = 20000
        r = native.query_walks(g, v, 7, 11, s, 0, s, t, W)
        for vals, want in ((r["dep_a"] / d[s], Lvi[s, s]), (r["dep_b"] / d[t], Lvi[s, t]),
                           (r["norm_len"], Lvi[s].sum())):
            z = (vals.mean() - want) / (vals.std(ddof=1) / math.sqrt(W))
            assert abs(z) < 4.5


def test_sub_streams_and_qid_differ():
    g = graph("grid", 3, 3)
    a = native.query_walks(g, 0, 1, 5, 8, 0, 8, 4, 50)
    b = native.query_walks(g, 0, 1, 5, 8, 1, 8, 4, 50)
    c = native.query_walks(g, 0, 1, 6, 8, 0, 8, 4, 50)
    assert not np.array_equal(a["len"], b["len"]) and not np.array_equal(a["len"], c["len"])


def test_walk_from_root_is_empty():
    g = graph("grid", 3, 3)
    r = native.query_walks(g, 4, 1, 0, 4, 0, 4, 2, 10)
    assert (r["len"] == 0).all() and (r["dep_a"] == 0).all() and (r["norm_len"] == 0).all()


def test_query_assembly_exact_with_expectations():
    g = graph("grid", 3, 4)
    v = 5
    L = dense.laplacian(g)
    Ld = dense.pinv_eigh(L)
    Lvi = dense.lv_inv(L, v)
    n = g.n
    tr_lv, s_lv = np.trace(Lvi), Lvi.sum()
    for u in range(n):
        # a single "walk" carrying the exact expectations
        c, ld, _ = estimators.closeness_query([Lvi[u, u] * g.deg[u]], [Lvi[u].sum()], g.deg[u], n, tr_lv, s_lv)
        assert ld == pytest.approx(Ld[u, u], abs=1e-12)
        assert c == pytest.approx(dense.closeness(Ld)[u], rel=1e-12)
    for s, t in ((0, 11), (3, 8), (v, 2)):
        r, _ = estimators.resistance_query([Lvi[s, s] * g.deg[s]], [Lvi[s, t] * g.deg[t]],
                                           [Lvi[t, t] * g.deg[t]], [Lvi[t, s] * g.deg[s]], g.deg[s], g.deg[t])
        assert r == pytest.approx(dense.resistance(Ld, s, t), abs=1e-12)


def test_globals_from_exact_expectations():
    g = graph("grid", 3, 4)
    v = 1
    e = dense.expected_counts(g, v)
    Lvi = dense.lv_inv(dense.laplacian(g), v)
    tr, s = estimators.globals_from_counts(e["draws"], e["visits_uniform"], 1, g.deg, v)
    assert tr == pytest.approx(np.trace(Lvi), rel=1e-12) and s == pytest.approx(Lvi.sum(), rel=1e-12)


def test_sampled_queries_within_tolerance_er256():
    g = er256()
    v = csr.landmark(g)
    L = dense.laplacian(g)
    Ld = dense.pinv_eigh(L)
    Lvi = dense.lv_inv(L, v)
    n = g.n
    tr_lv, s_lv = np.trace(Lvi), Lvi.sum()
    for qid, u in enumerate((3, 77, 200)):
        r = native.query_walks(g, v, 1, qid, u, 0, u, u, 4096)
        c, ld, se = estimators.closeness_query(r["dep_a"], r["norm_len"], g.deg[u], n, tr_lv, s_lv)
        assert abs(ld - Ld[u, u]) < 4 * se
    s_, t_ = 10, 150
    fs = native.query_walks(g, v, 1, 9, s_, 0, s_, t_, 4096)
    ft = native.query_walks(g, v, 1, 9, t_, 1, t_, s_, 4096)
    r, se = estimators.resistance_query(fs["dep_a"], fs["dep_b"], ft["dep_a"], ft["dep_b"], g.deg[s_], g.deg[t_])
    assert abs(r - dense.resistance(Ld, s_, t_)) < 4 * se
