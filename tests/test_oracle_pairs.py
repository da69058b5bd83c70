"""Pins for the oracle's loop-included paths from node pairs (Sec. 3.4, the
loop-erased-walk interpretation of L_v^{-1}) and the entries and resistances
assembled from them (r(s,t) of Sec. 2):

- a star rooted at its centre, where every path is one move and the
  resistances are exact;
- the path from s equals the first walk of a Wilson sample that starts at s
  (read from the Wilson oracle's own trajectory);
- every departure a path makes uses an entry that the Wilson sample drew;
- the expectations against the dense grounded inverse and pseudo-inverse;
- the closed forms of paths, cycles and complete graphs;
- the exact identities of equal, swapped and root pairs, and sample splitting;
- whole rows of L_v^{-1} (departures per node on the paths from given
  sources): equal to the pair counts where both exist, exact on a star,
  and against the dense grounded inverse and hitting times.
"""
import math

import numpy as np

from oracle import csr, dense, estimators, native
from tests.oracle_fixtures import er256, graph


def _entries(g, V, omega, s, t):
    return estimators.pair_entries(V, omega, g.deg[np.asarray(s)], g.deg[np.asarray(t)])


def test_star_rooted_at_centre_is_exact():
    g = graph("star", 7)
    s = np.array([1, 2, 0, 5, 0])
    t = np.array([2, 6, 3, 5, 0])
    omega = 300
    V = native.pair_paths(g, 0, omega, 3, s, t, B=4)
    tot = V.sum(0)
    # a leaf departs once, to the root; the root departs never
    exp = np.array([[1, 0, 1, 0], [1, 0, 1, 0], [0, 0, 1, 0], [1, 1, 1, 1], [0, 0, 0, 0]]) * omega
    assert np.array_equal(tot, exp)
    e = _entries(g, V, omega, s, t)
    np.testing.assert_array_equal(e["r"], [2.0, 2.0, 1.0, 0.0, 0.0])
    np.testing.assert_array_equal(e["r_se"], 0.0)
    np.testing.assert_array_equal(e["lv_st"], [0.0, 0.0, 0.0, 1.0, 0.0])


def test_path_is_the_first_walk_of_a_wilson_sample():
    """Started first, Wilson's walk from s reads the stacks from the bottom,
    which is the loop-included path from s (Fig. 1(d))."""
    for g, seed in ((graph("barabasi_albert", 40, 2, 1), 5), (graph("grid", 5, 6), 6), (er256(), 7)):
        v = csr.landmark(g)
        rng = np.random.default_rng(seed)
        for _ in range(12):
            i = int(rng.integers(0, 1000))
            s = int(rng.integers(0, g.n))
            if s == v:
                continue
            t = int(rng.integers(0, g.n))
            w = native.wilson_ordered(g, v, i, seed, np.array([s]), trace_cap=1 << 16)
            walk = w["trace"][:-1]                     # the draws' nodes; the last entry is the stop (v)
            assert w["trace"][-1] == v and len(walk) == w["total"]
            V = native.pair_paths(g, v, 1, seed, [s], [t], sample_begin=i, omega_total=i + 1)
            assert V[0, 0, 0] == np.count_nonzero(walk == s)
            assert V[0, 0, 1] == (np.count_nonzero(walk == t) if t != v else 0)


def test_paths_use_only_drawn_stack_entries():
    g = graph("barabasi_albert", 60, 2, 2)
    v = csr.landmark(g)
    rng = np.random.default_rng(0)
    s = rng.integers(0, g.n, 16)
    t = rng.integers(0, g.n, 16)
    for i in range(40):
        V = native.pair_paths(g, v, 1, 9, s, t, sample_begin=i, omega_total=i + 1)[0]
        k = native.wilson(g, v, i + 1, 9, sample_begin=i, n_samples=1, keep=[i])["draws"][0]
        k = k.astype(np.int64)
        k[v] = 0
        assert (V[:, 0] <= k[s]).all() and (V[:, 1] <= k[t]).all()
        assert (V[:, 2] <= k[t]).all() and (V[:, 3] <= k[s]).all()


def test_expectations_against_dense_inverse():
    g = graph("barabasi_albert", 30, 2, 3)
    v = csr.landmark(g)
    L = dense.laplacian(g)
    G = dense.walk_green(L, v)                         # expected departures from u of a walk from s
    Ld = dense.pinv_eigh(L)
    rng = np.random.default_rng(1)
    s = rng.integers(0, g.n, 24)
    t = rng.integers(0, g.n, 24)
    omega, B = 1 << 15, 64
    V = native.pair_paths(g, v, omega, 11, s, t, B=B)
    mean = V.sum(0) / omega
    sizes = estimators.block_sizes(omega, B)
    se = (V / sizes[:, None, None]).std(0, ddof=1) / math.sqrt(B)
    exp = np.stack([G[s, s], G[s, t], G[t, t], G[t, s]], axis=1)
    live = se > 0
    z = (mean[live] - exp[live]) / se[live]
    assert np.abs(z).max() < 5.0 and (np.abs(z) < 3).mean() > 0.97
    assert np.array_equal(exp == 0, mean == 0)         # zero exactly where the walk cannot depart
    e = _entries(g, V, omega, s, t)
    r_true = np.array([dense.resistance(Ld, a, b) for a, b in zip(s, t)])
    ok = e["r_se"] > 0
    zr = (e["r"][ok] - r_true[ok]) / e["r_se"][ok]
    assert np.abs(zr).max() < 4.5
    np.testing.assert_allclose(e["r"][~ok], r_true[~ok], atol=1e-12)
    Lvi = dense.lv_inv(L, v)
    np.testing.assert_allclose(e["lv_st"], Lvi[s, t], rtol=0.08, atol=0.01)


def test_resistance_closed_forms():
    cases = [
        (graph("path", 10), [(0, 9), (2, 7), (1, 1), (4, 5)], lambda a, b, n: abs(a - b)),
        (graph("cycle", 12), [(0, 6), (3, 4), (2, 11), (5, 9)], lambda a, b, n: (abs(a - b) * (n - abs(a - b))) / n),
        (graph("complete", 8), [(0, 1), (3, 7), (6, 2)], lambda a, b, n: (2.0 / n) if a != b else 0.0),
    ]
    for g, pairs, f in cases:
        v = csr.landmark(g)
        s = np.array([p[0] for p in pairs])
        t = np.array([p[1] for p in pairs])
        omega = 1 << 14
        e = _entries(g, native.pair_paths(g, v, omega, 2, s, t, B=32), omega, s, t)
        for j, (a, b) in enumerate(pairs):
            want = f(a, b, g.n)
            if a == b:
                assert e["r"][j] == 0.0
            else:
                assert abs(e["r"][j] - want) < 4.5 * e["r_se"][j], (a, b, e["r"][j], want)


def test_pair_identities_and_splitting():
    g = er256()
    v = csr.landmark(g)
    rng = np.random.default_rng(4)
    s = rng.integers(0, g.n, 20)
    t = rng.integers(0, g.n, 20)
    s[0] = t[0] = 17                                   # equal pair
    s[1], t[1] = v, 33                                 # pair with the root
    omega = 96
    V = native.pair_paths(g, v, omega, 5, s, t, B=3)
    Vsw = native.pair_paths(g, v, omega, 5, t, s, B=3)
    assert np.array_equal(Vsw, V[:, :, [2, 3, 0, 1]])
    assert V[:, 0, 0].tolist() == V[:, 0, 1].tolist() == V[:, 0, 2].tolist() == V[:, 0, 3].tolist()
    assert (V[:, 1, [0, 1, 3]] == 0).all()
    e = _entries(g, V, omega, s, t)
    assert e["r"][0] == 0.0
    assert e["r"][1] == e["lv_tt"][1]
    a = native.pair_paths(g, v, 40, 5, s, t, B=3, sample_begin=0, omega_total=omega)
    b = native.pair_paths(g, v, 56, 5, s, t, B=3, sample_begin=40, omega_total=omega)
    assert np.array_equal(a + b, V)


def test_rows_agree_with_pair_paths_exactly():
    """The row counts of the path from s at s and at t are the pair counts V0
    and V1 of the pair (s, t) (two separately written oracle loops)."""
    g = er256()
    v = csr.landmark(g)
    rng = np.random.default_rng(8)
    s = rng.integers(0, g.n, 12)
    t = rng.integers(0, g.n, 12)
    s[0] = v
    Y = native.lv_rows(g, v, 200, 6, s, B=4)
    V = native.pair_paths(g, v, 200, 6, s, t, B=4)
    j = np.arange(len(s))
    assert np.array_equal(Y[:, j, s], V[:, :, 0]) and np.array_equal(Y[:, j, t], V[:, :, 1])
    assert (Y[:, :, v] == 0).all() and (Y[:, 0, :] == 0).all()    # no departures from v; the row of v is zero


def test_rows_star_and_dense_expectations():
    g = graph("star", 7)
    Y = native.lv_rows(g, 0, 50, 2, [3, 0])
    assert Y[0, 0, 3] == 50 and Y[0, 0].sum() == 50 and Y[0, 1].sum() == 0
    g = graph("barabasi_albert", 30, 2, 4)
    v = csr.landmark(g)
    L = dense.laplacian(g)
    G = dense.walk_green(L, v)
    src = np.array([0, 5, 17, 29])
    omega, B = 1 << 14, 32
    Y = native.lv_rows(g, v, omega, 3, src, B=B)
    sizes = estimators.block_sizes(omega, B)
    mean = Y.sum(0) / omega
    se = (Y / sizes[:, None, None]).std(0, ddof=1) / math.sqrt(B)
    live = se > 0
    z = (mean[live] - G[src][live]) / se[live]
    assert np.abs(z).max() < 5.0 and (np.abs(z) < 3).mean() > 0.97
    assert np.array_equal(G[src] == 0, mean == 0)
    # row sums are path lengths: their expectation is the hitting time of v
    h = G[src].sum(1)
    tot = Y.sum(2)                                     # [B][sources]
    zt = (tot.sum(0) / omega - h) / ((tot / sizes[:, None]).std(0, ddof=1) / math.sqrt(B))
    assert np.abs(zt).max() < 4.0
    est = estimators.lv_rows(Y, omega, g.deg, v)
    Lvi = dense.lv_inv(L, v)
    np.testing.assert_allclose(est, Lvi[src], rtol=0.1, atol=0.02)
