"""SpanTree estimators on the GPU (Alg. 1, Alg. 3) against the oracle: the
per-block sums X1, X2 and the per-sample Kemeny terms s1, s2 are bit-exact
(same Wilson trees, integer flows), the FP64 assembly agrees to 1e-12, and
the estimates sit within their standard errors of the dense truth."""
import numpy as np
import pytest

from oracle import csr, dense, estimators, native
from tests.gpu_common import ba_edges, both, er256_edges, log, small_cases

pytestmark = pytest.mark.gpu


def _oracle(og, root, omega, seed, B=1, begin=0, total=None):
    total = total or begin + omega
    X1 = np.zeros((B, og.n), np.int64)
    X2 = np.zeros((B, og.n), np.int64)
    for b in range(B):
        lo = max(begin, -(-b * total // B))
        hi = min(begin + omega, -(-(b + 1) * total // B))
        if hi > lo:
            r = native.spantree(og, root, hi - lo, seed, 1, sample_begin=lo)
            X1[b], X2[b] = r["X1"], r["X2"]
    k = native.spantree(og, root, omega, seed, 2, sample_begin=begin)
    return dict(X1=X1, X2=X2, s1=k["s1"], s2=k["s2"])


def _same(a, b):
    for k in ("X1", "X2", "s1", "s2"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("mode,group", [(2, 0), (3, 4), (1, 0)])
def test_spantree_small_graphs_bit_exact(mode, group):
    for name, n, s, d in small_cases():
        og, hg = both(n, s, d)
        for root in sorted({0, csr.landmark(og), og.n - 1}):
            log(f"spantree {name} root {root} mode {mode}")
            got = hg.spantree(120, 4, root, B=3, mode=mode, group=group, pool=9)
            _same(got, _oracle(og, root, 120, 4, B=3))


def test_spantree_er256_workload_bit_exact():
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    log("spantree er256")
    got = hg.spantree(1 << 14, 1, root, B=64)
    _same(got, _oracle(og, root, 1 << 14, 1, B=64))


def test_spantree_rounds_and_resume():
    """More samples than slots (several Wilson + SpanTree rounds), and a run
    split in two halves."""
    n, s, d = ba_edges(20_000, 3, 4)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    log("spantree ba20k rounds")
    full = hg.spantree(50, 2, root, B=5, pool=7)
    _same(full, _oracle(og, root, 50, 2, B=5))
    a = hg.spantree(20, 2, root, B=5, sample_begin=0, n_total=50, pool=3)
    b = hg.spantree(30, 2, root, B=5, sample_begin=20, n_total=50, mode=3, group=8)
    assert np.array_equal(a["X1"] + b["X1"], full["X1"]) and np.array_equal(a["X2"] + b["X2"], full["X2"])
    assert np.array_equal(np.concatenate([a["s1"], b["s1"]]), full["s1"])


def test_spantree_estimates_match_oracle_and_dense_truth():
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega, B = 1 << 13, 64
    e = hg.spantree_estimate(omega, 1, root, B=B)
    o = _oracle(og, root, omega, 1, B=B)
    diag, se = estimators.spantree_diag_blocks(o["X1"], o["X2"], omega, og.n)
    np.testing.assert_allclose(e["diag"], diag, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(e["diag_se"], se, rtol=1e-9)
    c, _ = estimators.closeness(diag)
    np.testing.assert_allclose(e["closeness"], c, rtol=1e-12)
    k, kse = estimators.spantree_kemeny(o["s1"], o["s2"], og.nnz)
    assert e["kemeny"][0] == pytest.approx(k, rel=1e-12) and e["kemeny_se"][0] == pytest.approx(kse, rel=1e-9)
    # statistical tolerance against the dense pseudo-inverse and Kemeny's constant
    L = dense.laplacian(og)
    z = (e["diag"] - np.diag(dense.pinv_eigh(L))) / e["diag_se"]
    assert np.max(np.abs(z)) < 4.6 and np.mean(np.abs(z) < 3) >= 0.97
    assert abs(e["kemeny"][0] - dense.kemeny_spectral(og)) < 3 * e["kemeny_se"][0]


def test_spantree_full_size_sampled_trees_bit_exact():
    """The mid workload (Barabasi-Albert n = 100,000, m = 5, root = max
    degree): the sums of 16 trees equal the oracle's."""
    n, s, d = ba_edges(100_000, 5, 0)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    log("spantree ba100k")
    got = hg.spantree(16, 1, root, B=2)
    _same(got, _oracle(og, root, 16, 1, B=2))


def test_spantree_argument_errors():
    from paper_2311_10290_amd import LapError
    n, s, d = er256_edges()
    _, hg = both(n, s, d)
    with pytest.raises(LapError):
        hg.spantree(0, 1)
    with pytest.raises(LapError):
        hg.spantree(10, 1, root=999)


def test_spantree_sample_bounds():
    """Thm. 3 and Thm. 4 sample sizes: the BFS depth from v against the
    oracle's BFS tree, and the two bounds on a path, a star and the small ER
    workload."""
    import math
    from paper_2311_10290_amd import LapError
    import graphgen as gg
    cases = [("path", 9, gg.path(9)), ("star", 7, gg.star(7))]
    n, s, d = er256_edges()
    cases.append(("er256", n, (s, d)))
    for name, n, (s, d) in cases:
        og, hg = both(n, s, d)
        root = csr.landmark(og)
        par = native.bfs_tree(og, root)
        depth = 0
        for u in range(og.n):
            k, x = 0, u
            while x != root:
                x = int(par[x])
                k += 1
            depth = max(depth, k)
        m = og.nnz / 2
        w1, d1 = hg.spantree_sample_bound(1, 0.05, 0.01)
        w2, d2 = hg.spantree_sample_bound(2, 10.0, 0.1, root=root)
        assert d1 == d2 == depth, name
        assert w1 == math.ceil(32 * depth ** 2 * math.log(2 * og.n / 0.01) / 0.05 ** 2)
        assert w2 == math.ceil(8 * m * m * depth ** 2 * math.log(2 / 0.1) / 10.0 ** 2)
    with pytest.raises(LapError):
        hg.spantree_sample_bound(3, 0.1, 0.1)
    with pytest.raises(LapError):
        hg.spantree_sample_bound(1, 0.0, 0.1)
    with pytest.raises(LapError):
        hg.spantree_sample_bound(1, 0.1, 1.0)
