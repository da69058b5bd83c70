"""Pins for the FP64 dense ground truth: closed forms (K_n, cycles, paths,
stars, trees), the paper's worked flow examples (Figs. 3 and 4), the
Moore-Penrose conditions, and the paper's identities (Thm. 1 and the
element-wise equations, root invariance, the Kemeny lemma of Sec. 5, the
closeness formula)."""
import numpy as np
import pytest

from oracle import dense
from tests.oracle_fixtures import er256, graph, read_golden


def test_two_pinv_routes_agree_and_are_moore_penrose():
    for g in (graph("diamond"), graph("grid", 3, 4), graph("barabasi_albert", 40, 2, 1)):
        L = dense.laplacian(g)
        A, B = dense.pinv_eigh(L), dense.pinv_inverse(L)
        assert np.allclose(A, B, atol=1e-10, rtol=0)
        assert np.allclose(L @ A @ L, L, atol=1e-10)
        assert np.allclose(A @ L @ A, A, atol=1e-10)
        assert np.allclose(A.sum(1), 0.0, atol=1e-10)          # rows of L^dagger sum to 0
        assert np.allclose(A, A.T, atol=1e-12)


def test_er256_routes_agree():
    g = er256()
    L = dense.laplacian(g)
    assert np.allclose(dense.pinv_eigh(L), dense.pinv_inverse(L), atol=1e-10, rtol=0)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 13])
def test_complete_graph_closed_forms(n):
    g = graph("complete", n)
    Ld = dense.pinv_eigh(dense.laplacian(g))
    assert dense.kemeny_spectral(g) == pytest.approx((n - 1) ** 2 / n, rel=1e-12)  # Sec. 2 definition
    for s in range(n):
        for t in range(s + 1, n):
            assert dense.resistance(Ld, s, t) == pytest.approx(2.0 / n, rel=1e-12)


@pytest.mark.parametrize("n", [3, 4, 7, 10])
def test_cycle_closed_forms(n):
    g = graph("cycle", n)
    Ld = dense.pinv_eigh(dense.laplacian(g))
    assert dense.kemeny_spectral(g) == pytest.approx((n * n - 1) / 6.0, rel=1e-12)
    for s in range(n):
        for t in range(n):
            k = (t - s) % n
            assert dense.resistance(Ld, s, t) == pytest.approx(k * (n - k) / n, abs=1e-12)


def test_path_star_tree_resistances():
    for n in (2, 5, 9):
        Ld = dense.pinv_eigh(dense.laplacian(graph("path", n)))
        for s in range(n):
            for t in range(n):
                assert dense.resistance(Ld, s, t) == pytest.approx(abs(s - t), abs=1e-12)
    Ld = dense.pinv_eigh(dense.laplacian(graph("star", 6)))
    assert dense.resistance(Ld, 0, 3) == pytest.approx(1.0)
    assert dense.resistance(Ld, 2, 5) == pytest.approx(2.0)


def test_diamond_worked_examples():
    g = graph("diamond")
    L = dense.laplacian(g)
    Ld = dense.pinv_eigh(L)
    rows = read_golden("diamond.txt")
    want = np.array([[float(x) for x in r.split()] for t, r in rows if t == "ldagger16"])
    assert np.allclose(16 * Ld, want, atol=1e-12)
    wvs = float([r for t, r in rows if t == "weighted_voltage_sum"][0])
    kem = float([r for t, r in rows if t == "kemeny"][0])
    for v in (2, 3):     # landmark = a degree-2 node, as in Fig. 4
        d = np.diag(L).copy()
        dv = d.copy()
        dv[v] = 0
        Lvi = dense.lv_inv(L, v)
        assert dv @ Lvi @ dv / d.sum() == pytest.approx(wvs, abs=1e-12)
        assert np.trace(dense.walk_green(L, v)) == pytest.approx(wvs + kem, abs=1e-12)
    assert dense.kemeny_spectral(g) == pytest.approx(kem, abs=1e-12)
    assert np.allclose(dense.kemeny_hitting(g), kem, atol=1e-12)


@pytest.mark.parametrize("which", ["diamond", "grid", "ba"])
def test_thm1_and_elementwise_identities_every_root(which):
    g = {"diamond": lambda: graph("diamond"), "grid": lambda: graph("grid", 3, 3),
         "ba": lambda: graph("barabasi_albert", 25, 2, 3)}[which]()
    L = dense.laplacian(g)
    Ld = dense.pinv_eigh(L)
    for v in range(g.n):
        Lvi = dense.lv_inv(L, v)
        assert np.allclose(dense.ldagger_thm1(Lvi, v), Ld, atol=1e-10)        # Thm. 1, root invariance
        for s in range(g.n):
            for t in range(g.n):
                assert dense.ldagger_entry(Lvi, v, s, t) == pytest.approx(Ld[s, t], abs=1e-10)
        assert dense.kemeny_lemma(L, v) == pytest.approx(dense.kemeny_spectral(g), rel=1e-10)


def test_kemeny_definitions_agree_er256():
    g = er256()
    L = dense.laplacian(g)
    k = dense.kemeny_spectral(g)
    assert np.allclose(dense.kemeny_hitting(g), k, rtol=1e-9)
    for v in (0, 17, 245):
        assert dense.kemeny_lemma(L, v) == pytest.approx(k, rel=1e-10)


def test_closeness_is_inverse_mean_resistance():
    g = graph("grid", 3, 4)
    Ld = dense.pinv_eigh(dense.laplacian(g))
    c = dense.closeness(Ld)
    for u in range(g.n):
        tot = sum(dense.resistance(Ld, u, w) for w in range(g.n))
        assert c[u] == pytest.approx((g.n - 1) / tot, rel=1e-12)


def test_walk_green_counts_visits_by_linear_system():
    # Lemma 1: (I - P_v)^{-1}_{su} is the expected number of departures from u;
    # check against h(s,v) by first-step analysis on a path, h(s,v) = (v-s)(v+s) for v at the end
    n = 6
    g = graph("path", n)
    L = dense.laplacian(g)
    N = dense.walk_green(L, n - 1)
    for s in range(n - 1):
        assert N[s].sum() == pytest.approx((n - 1 - s) * (n - 1 + s), rel=1e-12)


def test_kirchhoff_index_closed_forms_and_trace_identity():
    from oracle import estimators
    for n in (3, 6, 9):
        Ld = dense.pinv_eigh(dense.laplacian(graph("complete", n)))
        assert dense.kirchhoff_pairs(Ld) == pytest.approx(n - 1, rel=1e-12)            # r = 2/n on every pair
        Ld = dense.pinv_eigh(dense.laplacian(graph("path", n)))
        assert dense.kirchhoff_pairs(Ld) == pytest.approx((n ** 3 - n) / 6, rel=1e-12)  # sum of |i-j|
        Ld = dense.pinv_eigh(dense.laplacian(graph("cycle", n)))
        assert dense.kirchhoff_pairs(Ld) == pytest.approx((n ** 3 - n) / 12, rel=1e-12)
    for g in (graph("grid", 3, 4), graph("barabasi_albert", 30, 2, 7)):
        Ld = dense.pinv_eigh(dense.laplacian(g))
        assert estimators.kirchhoff(np.diag(Ld)) == pytest.approx(dense.kirchhoff_pairs(Ld), rel=1e-10)


def test_rw_betweenness_closed_forms_and_farness_identity():
    """The random-walk betweenness formula quoted at the end of Sec. 5,
    c_b(u) = 1/n + Tr/((n-1)(Tr + n L^dagger_uu)), pinned without re-typing
    it.  Tr + n L^dagger_uu is the farness sum_v r(u,v) and Tr is the
    Kirchhoff index over n, so the formula is fixed by resistances alone:
    - K_n: r = 2/n on every pair, farness 2(n-1)/n, Tr (n-1)/n, so
      c_b = 1/n + 1/(2(n-1)) at every node;
    - star with n nodes: centre-leaf r = 1, leaf-leaf r = 2, Tr (n-1)^2/n;
      farness n-1 at the centre (c_b = 2/n) and 2n-3 at a leaf
      (c_b = 1/n + (n-1)/(n(2n-3)));
    - any graph: the value from the diagonal of the eigen-decomposition
      pseudo-inverse equals 1/n + (Kf/n)/((n-1) farness(u)), with Kf and the
      farness summed over resistances of the other route, (L + 11^T/n)^-1."""
    from oracle import estimators
    for n in (4, 7, 10):
        Ld = dense.pinv_eigh(dense.laplacian(graph("complete", n)))
        np.testing.assert_allclose(estimators.rw_betweenness(np.diag(Ld)), 1 / n + 1 / (2 * (n - 1)), rtol=1e-12)
        g = graph("star", n)
        Ld = dense.pinv_eigh(dense.laplacian(g))
        cb = estimators.rw_betweenness(np.diag(Ld))
        centre = int(np.argmax(g.deg))
        want = np.full(n, 1 / n + (n - 1) / (n * (2 * n - 3)))
        want[centre] = 2 / n
        np.testing.assert_allclose(cb, want, rtol=1e-12)
    for g in (graph("diamond"), graph("grid", 3, 4), graph("barabasi_albert", 30, 2, 7)):
        n = g.n
        L = dense.laplacian(g)
        cb = estimators.rw_betweenness(np.diag(dense.pinv_eigh(L)))
        Li = dense.pinv_inverse(L)
        R = np.array([[dense.resistance(Li, s, t) for t in range(n)] for s in range(n)])
        kf = R.sum() / 2
        np.testing.assert_allclose(cb, 1 / n + (kf / n) / ((n - 1) * R.sum(1)), rtol=1e-10)
