"""Parity of the HIP path against the oracle (bit-exact integer counts,
FP64 estimates within 1e-12 relative), through the C ABI."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr, dense, estimators, native
from tests.gpu_common import ba_edges, both, er256_edges, log, small_cases

pytestmark = pytest.mark.gpu

MODES = [1, 2, 4]       # LAP_MODE_LANE, LAP_MODE_WAVE, LAP_MODE_LDS


def _oracle_counts(og, root, omega, seed, B=1, keep=(), begin=0, total=None, uniform=True, pi=True):
    total = total or begin + omega
    w = native.wilson(og, root, total, seed, sample_begin=begin, n_samples=omega, B=B, keep=keep)
    out = dict(Y1=w["Y1"], y1=w["y1"], next=w["next"], draws=w["draws"])
    if uniform:
        a = native.absorbed(og, root, omega, seed, 1, walk_begin=begin, omega_total=total, B=B)
        out["Y2"], out["len_uniform"] = a["Y2"], a["len"]
    if pi:
        a = native.absorbed(og, root, omega, seed, 2, walk_begin=begin, omega_total=total, want_y2=False)
        out["len_pi"] = a["len"]
    return out


def _same(a, b, keys):
    for k in keys:
        assert a[k] is not None and b[k] is not None, k
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_csr_matches_oracle():
    cases = [("er256",) + er256_edges(), ("ba2000",) + ba_edges(2000, 3)]
    s, d = gg.rmat(12, 8, seed=4)
    cases.append(("rmat12", 4096, s, d))
    # above 2^20 edges the host builder splits the edges over threads: a
    # multigraph with self-loops and duplicates, and a disconnected one
    rng = np.random.default_rng(11)
    s = rng.integers(0, 150_000, 1_500_000).astype(np.int32)
    d = rng.integers(0, 150_000, 1_500_000).astype(np.int32)
    d[:1000] = s[:1000]
    s, d = np.concatenate([s, s[:5000]]), np.concatenate([d, d[:5000]])
    cases.append(("multigraph1.5M", 150_000, s, d))
    s = rng.integers(0, 400_000, 1_200_000).astype(np.int32)
    d = rng.integers(0, 400_000, 1_200_000).astype(np.int32)
    cases.append(("sparse1.2M", 400_000, s, d))
    for name, n, s, d in cases + small_cases():
        for dord in (False, True):
            log(f"csr {name} degree order {dord}")
            og, hg = both(n, s, d, keep_lcc=True, degree_order=dord)
            rp, col, old = hg.csr()
            assert hg.n == og.n and hg.nnz == og.nnz
            assert np.array_equal(rp, og.rp) and np.array_equal(col, og.col) and np.array_equal(old, og.old_ids)
            assert hg.max_deg_node == csr.landmark(og)


@pytest.mark.parametrize("mode", MODES)
def test_small_graphs_bit_exact(mode):
    for name, n, s, d in small_cases():
        og, hg = both(n, s, d)
        for root in sorted({0, csr.landmark(og), og.n - 1}):
            log(f"small {name} root {root} mode {mode}")
            omega = 300
            keep = [0, 1, 77, 299]
            got = hg.sample_forests(omega, 9, root, y2=True, y2_pi=True, B=4, keep=keep, mode=mode, pool=7)
            exp = _oracle_counts(og, root, omega, 9, B=4, keep=keep)
            _same(got, exp, ["Y1", "y1", "next", "draws", "Y2", "len_uniform", "len_pi"])


@pytest.mark.parametrize("mode", MODES)
def test_er256_workload_bit_exact(mode):
    """G(256, 0.05) seed 0 resampled until connected, root = max degree,
    2^14 samples with Philox seed 1, B = 64 blocks."""
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega = 1 << 14
    keep = [0, 5, 4095, 9999, omega - 1]
    log(f"er256 mode {mode}")
    got = hg.sample_forests(omega, 1, root, y2=True, y2_pi=True, B=64, keep=keep, mode=mode)
    exp = _oracle_counts(og, root, omega, 1, B=64, keep=keep)
    _same(got, exp, ["Y1", "y1", "next", "draws", "Y2", "len_uniform", "len_pi"])


@pytest.mark.parametrize("pool", [1, 3, 64, 1000])
def test_wave_pool_sizes_and_ragged_sample_counts(pool):
    n, s, d = ba_edges(3000, 2, 5)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega = 203
    log(f"pool {pool}")
    got = hg.sample_forests(omega, 3, root, y2=False, B=3, keep=[0, 202], mode=2, pool=pool)
    exp = _oracle_counts(og, root, omega, 3, B=3, keep=[0, 202], uniform=False, pi=False)
    _same(got, exp, ["Y1", "y1", "next", "draws"])


def test_schedule_rotation_does_not_change_counts():
    """Race check: rotating where the start scan begins changes which walker
    takes which start and the order of every claim, park and cycle pop; by
    Wilson's stack argument the counts and trees must not change."""
    n, s, d = ba_edges(3000, 3, 9)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    exp = _oracle_counts(og, root, 150, 4, B=2, keep=[0, 149], uniform=False, pi=False)
    for sched in (0, 1, 777, og.n - 1, 10**9 + 7):
        log(f"schedule {sched}")
        got = hg.sample_forests(150, 4, root, B=2, keep=[0, 149], mode=2, pool=50, schedule=sched)
        _same(got, exp, ["Y1", "y1", "next", "draws"])


def test_kernel_time_limit_is_reported_and_recovered():
    """A time limit forced from the host stops the kernels through their own
    bounded checks; the call reports LAP_ERANGE and the next call is exact."""
    from paper_2311_10290_amd import LapError
    n, s, d = ba_edges(200_000, 3, 2)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    with pytest.raises(LapError) as ei:
        hg.sample_forests(2048, 1, root, y2=True, timeout_s=1e-4)
    assert ei.value.code == -5
    got = hg.sample_forests(16, 1, root, y2=True, B=1)
    exp = _oracle_counts(og, root, 16, 1, B=1, pi=False)
    _same(got, exp, ["Y1", "y1", "Y2", "len_uniform"])


def test_resume_in_two_halves_equals_one_run():
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    full = hg.sample_forests(1000, 2, root, y2=True, B=8, mode=2)
    a = hg.sample_forests(400, 2, root, y2=True, B=8, sample_begin=0, n_total=1000, mode=2)
    b = hg.sample_forests(600, 2, root, y2=True, B=8, sample_begin=400, n_total=1000, mode=1)
    assert np.array_equal(a["Y1"] + b["Y1"], full["Y1"])
    assert np.array_equal(a["Y2"] + b["Y2"], full["Y2"])
    assert np.array_equal(np.concatenate([a["y1"], b["y1"]]), full["y1"])
    exp = _oracle_counts(og, root, 600, 2, B=8, begin=400, total=1000, pi=False)
    _same(b, exp, ["Y1", "y1", "Y2", "len_uniform"])


def test_stream_id_and_qid_change_the_stream():
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    a = hg.sample_forests(64, 1, -1, y2=True)
    b = hg.sample_forests(64, 1, -1, y2=True, stream_id=3)
    c = hg.sample_forests(64, 1, -1, y2=True, qid=5)
    assert not np.array_equal(a["y1"], b["y1"]) and not np.array_equal(a["y1"], c["y1"])


def test_estimates_match_oracle_assembly_and_dense_truth():
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega, B = 1 << 14, 64
    log("estimate er256")
    est = hg.estimate(omega, 1, root, B=B, lv=True)
    exp = _oracle_counts(og, root, omega, 1, B=B)
    diag, se = estimators.diag_ldagger_blocks(exp["Y1"], exp["Y2"], omega, og.deg)
    c, tr = estimators.closeness(diag)
    k, kse = estimators.kemeny(exp["y1"], exp["len_pi"])
    np.testing.assert_allclose(est["diag"], diag, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(est["diag_se"], se, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(est["closeness"], c, rtol=1e-12)
    np.testing.assert_allclose(est["trace"][0], tr, rtol=1e-12)
    np.testing.assert_allclose(est["kemeny"][0], k, rtol=1e-12)
    np.testing.assert_allclose(est["kemeny_se"][0], kse, rtol=1e-9)
    lv = exp["Y1"].sum(0) / (omega * og.deg)
    lv[root] = 0.0
    np.testing.assert_allclose(est["lv_diag"], lv, rtol=1e-12)
    # against the dense FP64 pseudo-inverse: statistical tolerance
    Ld = dense.pinv_eigh(dense.laplacian(og))
    z = (est["diag"] - np.diag(Ld)) / est["diag_se"]
    assert np.abs(z).max() < 4.6 and (np.abs(z) < 3).mean() >= 0.97
    assert abs(est["kemeny"][0] - dense.kemeny_spectral(og)) < 3 * est["kemeny_se"][0]


@pytest.mark.parametrize("B", [1, 2, 1024, 1025, 3000])
def test_assembly_over_block_counts(B):
    """The assembly keeps per-block constants in LDS for up to 1024 blocks and
    computes them per block beyond; one sample per block at B = omega."""
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega = 3000
    log(f"estimate er256 B={B}")
    est = hg.estimate(omega, 6, root, B=B, lv=True)
    exp = _oracle_counts(og, root, omega, 6, B=B)
    diag, se = estimators.diag_ldagger_blocks(exp["Y1"], exp["Y2"], omega, og.deg)
    c, tr = estimators.closeness(diag)
    np.testing.assert_allclose(est["diag"], diag, rtol=1e-12, atol=1e-15)
    if B > 1:
        np.testing.assert_allclose(est["diag_se"], se, rtol=1e-9, atol=1e-15)
    else:
        assert np.isnan(est["diag_se"]).all()
    np.testing.assert_allclose(est["closeness"], c, rtol=1e-12)
    np.testing.assert_allclose(est["trace"][0], tr, rtol=1e-12)
    lv = exp["Y1"].sum(0) / (omega * og.deg)
    lv[root] = 0.0
    np.testing.assert_allclose(est["lv_diag"], lv, rtol=1e-12)


@pytest.mark.parametrize("mode,group,pool", [(0, 0, 0), (2, 0, 7), (3, 4, 0), (1, 0, 300)])
def test_loop_included_estimates_match_oracle(mode, group, pool):
    """lap_estimate with the walk counts from the loop-included paths of the
    same Wilson samples (LAP_WALKS_LOOP): the samples run in rounds of the
    state slots (several rounds here), and every output equals the oracle's
    assembly of its Wilson counts and loop-included paths; at seed 1 the
    estimates meet the 1e-2 relative target against the dense pseudo-inverse."""
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega, B = 1 << 14, 64
    log(f"loop estimate er256 mode {mode} group {group} pool {pool}")
    est = hg.estimate(omega, 1, root, B=B, walks=1, mode=mode, group=group, pool=pool)
    w = native.wilson(og, root, omega, 1, B=B)
    l1 = native.loop_included(og, root, omega, 1, 1, B=B)
    l2 = native.loop_included(og, root, omega, 1, 2)
    diag, se = estimators.diag_ldagger_blocks(w["Y1"], l1["Y2"], omega, og.deg)
    c, tr = estimators.closeness(diag)
    k, kse = estimators.kemeny(w["y1"], l2["len"])
    np.testing.assert_allclose(est["diag"], diag, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(est["diag_se"], se, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(est["closeness"], c, rtol=1e-12)
    np.testing.assert_allclose(est["trace"][0], tr, rtol=1e-12)
    np.testing.assert_allclose(est["kemeny"][0], k, rtol=1e-12)
    np.testing.assert_allclose(est["kemeny_se"][0], kse, rtol=1e-9)
    Ld = dense.pinv_eigh(dense.laplacian(og))
    c_true = dense.closeness(Ld)
    assert abs(est["kemeny"][0] / dense.kemeny_spectral(og) - 1) < 1e-2
    assert np.max(np.abs(est["closeness"] - c_true) / c_true) < 1e-2


def test_loop_included_estimates_on_small_graphs():
    for name, n, s, d in small_cases():
        og, hg = both(n, s, d)
        root = csr.landmark(og)
        log(f"loop estimate {name}")
        est = hg.estimate(300, 4, root, B=4, walks=1, pool=7)
        w = native.wilson(og, root, 300, 4, B=4)
        l1 = native.loop_included(og, root, 300, 4, 1, B=4)
        l2 = native.loop_included(og, root, 300, 4, 2)
        diag, _ = estimators.diag_ldagger_blocks(w["Y1"], l1["Y2"], 300, og.deg)
        k, _ = estimators.kemeny(w["y1"], l2["len"])
        np.testing.assert_allclose(est["diag"], diag, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(est["kemeny"][0], k, rtol=1e-12, atol=1e-12)


def test_derived_outputs_match_oracle():
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    est = hg.estimate(2048, 5, root, B=8, derived=True)
    exp = _oracle_counts(og, root, 2048, 5, B=8)
    diag = estimators.diag_ldagger(exp["Y1"].sum(0), exp["Y2"].sum(0), 2048, og.deg)
    np.testing.assert_allclose(est["kirchhoff"][0], estimators.kirchhoff(diag), rtol=1e-12)
    np.testing.assert_allclose(est["rw_betweenness"], estimators.rw_betweenness(diag), rtol=1e-12)


def test_convenience_entry_points_agree():
    from paper_2311_10290_amd import diag_Ldagger, ecc, kemeny
    n, s, d = er256_edges()
    _, hg = both(n, s, d)
    est = hg.estimate(512, 4, -1, B=64)
    dd, se = diag_Ldagger(hg, 512, 4)
    np.testing.assert_array_equal(dd, est["diag"])
    np.testing.assert_array_equal(se, est["diag_se"])
    c, tr = ecc(hg, 512, 4)
    est1 = hg.estimate(512, 4, -1, B=1, se=False)
    np.testing.assert_array_equal(c, est1["closeness"])
    k, kse = kemeny(hg, 512, 4)
    assert k == est["kemeny"][0] and kse == est["kemeny_se"][0]


def test_degenerate_graphs():
    from paper_2311_10290_amd import Graph
    g1 = Graph(1, [], [])
    e = g1.estimate(8, 1, B=4)
    assert (e["diag"] == 0).all() and e["kemeny"][0] == 0.0 and (e["closeness"] == 0).all()
    og, hg = both(2, np.array([0]), np.array([1]))
    got = hg.sample_forests(50, 1, 0, y2=True, y2_pi=True, keep=[3])
    exp = _oracle_counts(og, 0, 50, 1, keep=[3])
    _same(got, exp, ["Y1", "y1", "Y2", "len_uniform", "len_pi", "next", "draws"])
    assert (got["y1"] == 1).all()              # one draw per sample: the only other node


def test_argument_errors():
    from paper_2311_10290_amd import LapError
    n, s, d = er256_edges()
    _, hg = both(n, s, d)
    for kw in [dict(root=256), dict(B=0), dict(keep=[5000]), dict(mode=7)]:
        args = dict(omega=100, seed=1)
        args.update(kw)
        with pytest.raises(LapError):
            hg.sample_forests(args.pop("omega"), args.pop("seed"), **args)
    with pytest.raises(LapError):
        hg.sample_forests(0, 1)


def test_profiling_counters():
    from paper_2311_10290_amd import prof_enable, prof_read, prof_reset
    n, s, d = er256_edges()
    _, hg = both(n, s, d)
    prof_reset()
    prof_enable(True)
    hg.estimate(256, 1)                 # automatic mode: the wave form
    hg.estimate(256, 1, mode=4)
    prof_enable(False)
    for name in ("wilson_wave", "wilson_lds"):
        ms, cnt = prof_read(name)
        assert cnt == 1 and ms > 0, name
    ms, cnt = prof_read("absorbed")
    assert cnt == 2 and ms > 0          # both walk kinds in one launch per call
    st = hg.last_stats()
    assert st["trees"] == 256 and st["wilson_steps"] > 0 and st["absorbed_steps"] > 0
