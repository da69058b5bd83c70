"""Loop-included paths from node pairs and from sources on the GPU against the
oracle: the per-block departure sums V and the row counts Y are bit-exact (the
same stack entries are read), with and without the Wilson run that checks
every entry was drawn, in every sampler form; the FP64 entries, rows and
resistances agree to 1e-12 and sit within their standard errors of the dense
truth."""
import numpy as np
import pytest

from oracle import csr, dense, estimators, native
from tests.gpu_common import ba_edges, both, er256_edges, log, small_cases

pytestmark = pytest.mark.gpu


def _pairs(n, root, k, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, k).astype(np.int32)
    t = rng.integers(0, n, k).astype(np.int32)
    s[0], t[0] = root, t[0]            # a pair with the root
    if k > 1:
        t[1] = s[1]                    # an equal pair
    return s, t


def _same(og, got, s, t, omega, seed, B, root, sample_begin=0, n_total=None):
    exp = native.pair_paths(og, root, omega, seed, s, t, B=B, sample_begin=sample_begin, omega_total=n_total)
    assert np.array_equal(got["V"], exp)
    e = estimators.pair_entries(exp, omega, og.deg[s], og.deg[t])
    np.testing.assert_allclose(got["r"], e["r"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(got["lv"], np.stack([e["lv_ss"], e["lv_st"], e["lv_tt"]], axis=1),
                               rtol=1e-12, atol=1e-15)
    if B > 1:
        np.testing.assert_allclose(got["r_se"], e["r_se"], rtol=1e-9, atol=1e-15)
    else:
        assert np.isnan(got["r_se"]).all()


@pytest.mark.parametrize("mode,group", [(2, 0), (3, 4), (1, 0)])
def test_pair_paths_small_graphs_bit_exact(mode, group):
    for name, n, src, dst in small_cases():
        og, hg = both(n, src, dst)
        for root in sorted({0, csr.landmark(og), og.n - 1}):
            s, t = _pairs(og.n, root, 9, root + 1)
            for check in (1, 0):
                log(f"pairs {name} root {root} mode {mode} check {check}")
                got = hg.pair_paths(s, t, 120, 4, root, B=3, check=check, mode=mode, group=group, pool=7)
                _same(og, got, s, t, 120, 4, 3, root)


def test_pair_paths_er256_workload_bit_exact_and_against_dense():
    n, src, dst = er256_edges()
    og, hg = both(n, src, dst)
    root = csr.landmark(og)
    s, t = _pairs(og.n, root, 256, 5)
    omega, B = 1 << 14, 64
    for check in (1, 0):
        log(f"pairs er256 check {check}")
        got = hg.pair_paths(s, t, omega, 1, root, B=B, check=check)
        _same(og, got, s, t, omega, 1, B, root)
    Ld = dense.pinv_eigh(dense.laplacian(og))
    truth = np.array([dense.resistance(Ld, a, b) for a, b in zip(s, t)])
    ok = got["r_se"] > 0
    z = (got["r"][ok] - truth[ok]) / got["r_se"][ok]
    assert np.abs(z).max() < 4.7 and (np.abs(z) < 3).mean() > 0.97
    np.testing.assert_allclose(got["r"][~ok], truth[~ok], atol=1e-12)


def test_pair_paths_mid_workload_bit_exact():
    """Barabasi-Albert n = 100,000, m = 5, root = max degree: 64 pairs over
    256 samples, with the Wilson check and without."""
    n, src, dst = ba_edges(100_000, 5, 0)
    og, hg = both(n, src, dst)
    root = csr.landmark(og)
    s, t = _pairs(og.n, root, 64, 6)
    for check in (1, 0):
        log(f"pairs ba100k check {check}")
        got = hg.pair_paths(s, t, 256, 1, root, B=8, check=check)
        _same(og, got, s, t, 256, 1, 8, root)
    log("pairs ba100k lanes 300")
    got = hg.pair_paths(s, t, 256, 1, root, B=8, check=0, lanes=300)
    _same(og, got, s, t, 256, 1, 8, root)


def test_pair_paths_many_pairs_few_samples_and_resume():
    """More paths than samples (several lanes per sample), and a run split
    in two sample ranges."""
    n, src, dst = ba_edges(5000, 3, 1)
    og, hg = both(n, src, dst)
    root = csr.landmark(og)
    s, t = _pairs(og.n, root, 3000, 7)
    log("pairs ba5k many pairs")
    got = hg.pair_paths(s, t, 3, 2, root, check=1)
    _same(og, got, s, t, 3, 2, 1, root)
    s, t = s[:50], t[:50]
    full = hg.pair_paths(s, t, 40, 2, root, B=4, pool=6)
    a = hg.pair_paths(s, t, 15, 2, root, B=4, sample_begin=0, n_total=40, check=0)
    b = hg.pair_paths(s, t, 25, 2, root, B=4, sample_begin=15, n_total=40, mode=3, group=2)
    assert np.array_equal(a["V"] + b["V"], full["V"])
    _same(og, full, s, t, 40, 2, 4, root)
    # few lanes: many launches, each lane's counters reused under new tags
    for lanes, check in ((7, 0), (64, 0), (5, 1), (100, 1)):
        log(f"pairs ba5k lanes {lanes} check {check}")
        got = hg.pair_paths(s, t, 40, 2, root, B=4, check=check, lanes=lanes, pool=6)
        assert np.array_equal(got["V"], full["V"])


def test_pair_paths_tables_that_fill_up_bit_exact():
    """Graphs with more nodes than a lane's table has words take the hashed
    form.  On these Erdos-Renyi graphs 6%, 24% and 31% of the paths meet
    more distinct nodes than a table allows and run again in the dense form
    (past a quarter, the rest of the call stays dense).  With few lanes the
    call takes many launches."""
    import graphgen as gg
    for n, deg, seed, lanes in ((20_000, 8, 0, 97), (30_000, 8, 2, 0), (40_000, 10, 4, 1000)):
        src, dst = gg.erdos_renyi(n, deg / n, seed)
        og, hg = both(n, src, dst, keep_lcc=True)
        root = csr.landmark(og)
        s, t = _pairs(og.n, root, 24, seed + 8)
        omega = 16
        # precondition: some of these paths outgrow a table (more than 12288 distinct nodes)
        big = 0
        for i in range(omega):
            for a in np.concatenate([s, t]):
                tr = native.loop_included_path(og.n, root, int(a), g=og, sample=i, seed=3, trace_cap=1 << 24)
                big += len(np.unique(tr[:-1])) > 12288
        assert big > 0
        for check in (0, 1):
            log(f"pairs er{n} lanes {lanes} check {check}")
            got = hg.pair_paths(s, t, omega, 3, root, B=4, check=check, lanes=lanes)
            _same(og, got, s, t, omega, 3, 4, root)


def _same_rows(og, got, src, omega, seed, B, root):
    exp = native.lv_rows(og, root, omega, seed, src, B=B)
    assert np.array_equal(got["Y"], exp)
    np.testing.assert_allclose(got["rows"], estimators.lv_rows(exp, omega, og.deg, root), rtol=1e-12, atol=0)


@pytest.mark.parametrize("mode,group", [(2, 0), (3, 4), (1, 0)])
def test_lv_rows_small_graphs_bit_exact(mode, group):
    for name, n, src, dst in small_cases():
        og, hg = both(n, src, dst)
        for root in sorted({0, csr.landmark(og), og.n - 1}):
            srcs = np.array(sorted({0, root, og.n - 1, og.n // 2}), np.int32)
            for check in (1, 0):
                log(f"rows {name} root {root} mode {mode} check {check}")
                got = hg.lv_rows(srcs, 90, 5, root, B=3, check=check, mode=mode, group=group, pool=7)
                _same_rows(og, got, srcs, 90, 5, 3, root)


def test_lv_rows_mid_workload_and_full_tables_bit_exact():
    """Rows on the mid workload (hashed tables) and on an Erdos-Renyi graph
    of 30,000 nodes where about a quarter of the paths outgrow their table:
    their departures are taken back out of the row before the dense form
    runs them again."""
    import graphgen as gg
    n, src, dst = ba_edges(100_000, 5, 0)
    og, hg = both(n, src, dst)
    root = csr.landmark(og)
    srcs = np.array([root, 0, 1, 77, 5000, 99_999], np.int32)
    for check, lanes in ((1, 0), (0, 0), (0, 300)):
        log(f"rows ba100k check {check} lanes {lanes}")
        got = hg.lv_rows(srcs, 64, 1, root, B=4, check=check, lanes=lanes)
        _same_rows(og, got, srcs, 64, 1, 4, root)
    src, dst = gg.erdos_renyi(30_000, 8 / 30_000, 2)
    og, hg = both(30_000, src, dst, keep_lcc=True)
    root = csr.landmark(og)
    srcs = np.random.default_rng(3).integers(0, og.n, 8).astype(np.int32)
    for check, lanes in ((0, 0), (1, 97)):
        log(f"rows er30k check {check} lanes {lanes}")
        got = hg.lv_rows(srcs, 16, 3, root, B=2, check=check, lanes=lanes)
        _same_rows(og, got, srcs, 16, 3, 2, root)


def test_pair_paths_argument_errors():
    from paper_2311_10290_amd import LapError
    n, src, dst = er256_edges()
    _, hg = both(n, src, dst)
    with pytest.raises(LapError):
        hg.pair_paths([], [], 10, 1)
    with pytest.raises(LapError):
        hg.pair_paths([0, 300], [1, 2], 10, 1)
    with pytest.raises(LapError):
        hg.pair_paths([0], [-1], 10, 1)
    with pytest.raises(LapError):
        hg.pair_paths([0], [1], 10, 1, lanes=-1)
    with pytest.raises(ValueError):
        hg.pair_paths([0, 1], [1], 10, 1)
    with pytest.raises(LapError):
        hg.lv_rows([], 10, 1)
    with pytest.raises(LapError):
        hg.lv_rows([256], 10, 1)
