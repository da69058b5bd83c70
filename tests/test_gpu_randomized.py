"""Randomised parity sweep: seeded random small graphs of several families,
random roots, sample counts, seeds, stream and query ids, sampler forms,
pools and scan rotations; every integer count must equal the oracle's.
By Wilson's stack argument no schedule may change a count, so this also
sweeps walker interleavings for races."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr, native
from tests.gpu_common import both, log

pytestmark = pytest.mark.gpu


def _graph(rng, i):
    kind = i % 4
    if kind == 0:
        n = int(rng.integers(20, 400))
        s, d, _ = gg.erdos_renyi_connected(n, float(rng.uniform(3.0, 9.0)) / n, int(rng.integers(1 << 30)))
        return n, s, d, False
    if kind == 1:
        n = int(rng.integers(20, 3000))
        s, d = gg.barabasi_albert(n, int(rng.integers(1, 5)), int(rng.integers(1 << 30)))
        return n, s, d, False
    if kind == 2:
        r, c = int(rng.integers(2, 30)), int(rng.integers(2, 30))
        s, d = gg.grid(r, c)
        return r * c, s, d, False
    scale = int(rng.integers(6, 12))
    s, d = gg.rmat(scale, 8, seed=int(rng.integers(1 << 30)))
    return 1 << scale, s, d, True


@pytest.mark.parametrize("case", range(12))
def test_random_graph_counts_bit_exact_lds_form(case):
    """The LDS lane form on random graphs it takes (at most 1024 nodes, columns
    and state in LDS), with random roots, seeds, stream and query ids and pools."""
    rng = np.random.default_rng(5000 + case)
    kind = case % 4
    if kind == 0:
        n = int(rng.integers(20, 1000))
        s, d, _ = gg.erdos_renyi_connected(n, float(rng.uniform(8.0, 14.0)) / n, int(rng.integers(1 << 30)))
    elif kind == 1:
        n = int(rng.integers(20, 1000))
        s, d = gg.barabasi_albert(n, int(rng.integers(1, 6)), int(rng.integers(1 << 30)))
    elif kind == 2:
        r, c = int(rng.integers(2, 32)), int(rng.integers(2, 32))
        s, d = gg.grid(r, c)
        n = r * c
    else:
        n = 1 << int(rng.integers(6, 11))
        s, d = gg.rmat(int(np.log2(n)), 8, seed=int(rng.integers(1 << 30)))
    og, hg = both(n, s, d, keep_lcc=kind == 3)
    assert og.n <= 1024 and 4 * ((og.n + 1) + (og.nnz + 1) // 2 + og.n * 16) <= 64 * 1024
    root = int(rng.integers(0, og.n)) if case % 2 else csr.landmark(og)
    omega = int(rng.integers(1, 400))
    seed = int(rng.integers(1 << 62))
    stream = int(rng.integers(0, 4))
    qid = int(rng.integers(0, 1 << 40))
    B = int(rng.integers(1, min(omega, 8) + 1))
    pool = int(rng.integers(0, 200))
    keep = sorted({0, omega - 1})
    log(f"random lds case {case}: n={og.n} nnz={og.nnz} root={root} omega={omega} pool={pool}")
    got = hg.sample_forests(omega, seed, root, B=B, keep=keep, mode=4, pool=pool, stream_id=stream, qid=qid)
    w = native.wilson(og, root, omega, seed, stream=stream, qid=qid, B=B, keep=keep)
    assert np.array_equal(got["Y1"], w["Y1"]) and np.array_equal(got["y1"], w["y1"])
    assert np.array_equal(got["next"], w["next"]) and np.array_equal(got["draws"], w["draws"])


@pytest.mark.parametrize("case", range(24))
def test_random_graph_counts_bit_exact(case):
    rng = np.random.default_rng(1000 + case)
    n, s, d, lcc = _graph(rng, case)
    og, hg = both(n, s, d, keep_lcc=lcc)
    root = int(rng.integers(0, og.n)) if case % 3 else csr.landmark(og)
    omega = int(rng.integers(1, 300))
    seed = int(rng.integers(1 << 62))
    stream = int(rng.integers(0, 4))
    qid = int(rng.integers(0, 1 << 40))
    B = int(rng.integers(1, min(omega, 8) + 1))
    mode, group = [(1, 0), (2, 0), (3, 2), (3, 4), (3, 8)][case % 5]
    pool = int(rng.integers(0, 50))
    sched = int(rng.integers(0, 1 << 31))
    keep = sorted({0, omega - 1})
    log(f"random case {case}: n={og.n} root={root} omega={omega} mode={mode}/{group} pool={pool}")
    got = hg.sample_forests(omega, seed, root, y2=True, y2_pi=True, B=B, keep=keep, mode=mode, group=group,
                            pool=pool, stream_id=stream, qid=qid, schedule=sched)
    w = native.wilson(og, root, omega, seed, stream=stream, qid=qid, B=B, keep=keep)
    a = native.absorbed(og, root, omega, seed, 1, stream=stream, qid=qid, B=B)
    p = native.absorbed(og, root, omega, seed, 2, stream=stream, qid=qid, want_y2=False)
    assert np.array_equal(got["Y1"], w["Y1"]) and np.array_equal(got["y1"], w["y1"])
    assert np.array_equal(got["next"], w["next"]) and np.array_equal(got["draws"], w["draws"])
    assert np.array_equal(got["Y2"], a["Y2"]) and np.array_equal(got["len_uniform"], a["len"])
    assert np.array_equal(got["len_pi"], p["len"])


def _pair_graph(rng, i):
    # every third case is large enough for the hashed form (more than 16384 nodes)
    if i % 3 == 2:
        if i % 2:
            n = int(rng.integers(17_000, 40_000))
            s, d = gg.barabasi_albert(n, int(rng.integers(2, 6)), int(rng.integers(1 << 30)))
            return n, s, d, False
        scale = 15
        s, d = gg.rmat(scale, 8, seed=int(rng.integers(1 << 30)))
        return 1 << scale, s, d, True
    return _graph(rng, i)


@pytest.mark.parametrize("case", range(18))
def test_random_pair_paths_bit_exact(case):
    """Node-pair paths (lap_pair_paths) on random graphs, roots, pairs, seeds,
    ids, block counts, sample ranges, lane caps, sampler forms and both check
    settings: the per-block sums equal the oracle's."""
    rng = np.random.default_rng(5000 + case)
    n, s, d, lcc = _pair_graph(rng, case)
    og, hg = both(n, s, d, keep_lcc=lcc)
    large = og.n > 16384
    # on the large graphs a low-degree root makes paths of ~2m/d_v steps: keep the landmark there
    root = int(rng.integers(0, og.n)) if (case % 4 and not large) else csr.landmark(og)
    P = int(rng.integers(1, 40))
    ps = rng.integers(0, og.n, P).astype(np.int32)
    pt = rng.integers(0, og.n, P).astype(np.int32)
    if P > 2:
        ps[0] = root
        pt[1] = ps[1]
    omega = int(rng.integers(1, 40))
    begin = int(rng.integers(0, 5))
    total = begin + omega + int(rng.integers(0, 5))
    B = int(rng.integers(1, min(total, 6) + 1))
    seed = int(rng.integers(1 << 62))
    stream = int(rng.integers(0, 4))
    qid = int(rng.integers(0, 1 << 40))
    mode, group = [(1, 0), (2, 0), (3, 2), (3, 4), (3, 8)][case % 5]
    check = case % 2
    lanes = [0, 1, 7, 64, 1000][int(rng.integers(0, 5))]
    if large:
        lanes = max(lanes, 64)
    log(f"random pair case {case}: n={og.n} root={root} pairs={P} omega={omega} begin={begin} "
        f"mode={mode}/{group} check={check} lanes={lanes}")
    got = hg.pair_paths(ps, pt, omega, seed, root, B=B, check=check, lanes=lanes, sample_begin=begin,
                        n_total=total, mode=mode, group=group, stream_id=stream, qid=qid)
    exp = native.pair_paths(og, root, omega, seed, ps, pt, stream=stream, qid=qid, sample_begin=begin,
                            omega_total=total, B=B)
    assert np.array_equal(got["V"], exp)


@pytest.mark.parametrize("case", range(9))
def test_random_lv_rows_bit_exact(case):
    """Whole rows (lap_lv_rows) on random graphs, roots, sources, seeds, ids,
    block counts, sample ranges, lane caps, sampler forms and both check
    settings: the row counts equal the oracle's."""
    rng = np.random.default_rng(7000 + case)
    n, s, d, lcc = _pair_graph(rng, case)
    og, hg = both(n, s, d, keep_lcc=lcc)
    large = og.n > 16384
    root = int(rng.integers(0, og.n)) if (case % 4 and not large) else csr.landmark(og)
    k = int(rng.integers(1, 12))
    src = rng.integers(0, og.n, k).astype(np.int32)
    src[0] = root if k > 1 else src[0]
    omega = int(rng.integers(1, 30))
    begin = int(rng.integers(0, 5))
    total = begin + omega + int(rng.integers(0, 5))
    B = int(rng.integers(1, min(total, 4) + 1))
    seed = int(rng.integers(1 << 62))
    stream = int(rng.integers(0, 4))
    qid = int(rng.integers(0, 1 << 40))
    mode, group = [(1, 0), (2, 0), (3, 2), (3, 4), (3, 8)][case % 5]
    check = (case + 1) % 2
    lanes = [0, 1, 7, 64, 1000][int(rng.integers(0, 5))]
    if large:
        lanes = max(lanes, 64)
    log(f"random rows case {case}: n={og.n} root={root} sources={k} omega={omega} begin={begin} "
        f"mode={mode}/{group} check={check} lanes={lanes}")
    got = hg.lv_rows(src, omega, seed, root, B=B, check=check, lanes=lanes, sample_begin=begin, n_total=total,
                     mode=mode, group=group, stream_id=stream, qid=qid)
    exp = native.lv_rows(og, root, omega, seed, src, stream=stream, qid=qid, sample_begin=begin,
                         omega_total=total, B=B)
    assert np.array_equal(got["Y"], exp)


@pytest.mark.parametrize("case", range(8))
def test_random_batches_bit_exact(case):
    """Batched launches (lap_batch_*) of random job lists: graph families and
    sizes, roots, sample counts, seeds, stream and query ids, pools, chunk
    sizes, eager or captured launches.  Every job's counts equal the oracle's
    for that job alone."""
    from paper_2311_10290_amd import Batch
    rng = np.random.default_rng(9000 + case)
    jobs, graphs = [], []
    for j in range(int(rng.integers(1, 13))):
        n, s, d, _ = _graph(rng, int(rng.integers(0, 4)))
        og = csr.build_csr(n, s, d, keep_lcc=True)
        root = -1 if rng.random() < 0.5 else int(rng.integers(0, og.n))
        jobs.append(dict(n=n, src=s, dst=d, keep_lcc=True, root=root, omega=int(rng.integers(1, 200)),
                         seed=int(rng.integers(1 << 62)), stream_id=int(rng.integers(0, 4)),
                         qid=int(rng.integers(0, 1 << 40))))
        graphs.append(og)
    pool = [0, 1, 3, 64, 500][int(rng.integers(0, 5))]
    chunk = [0, 1, 100, 5000, 1 << 20][int(rng.integers(0, 5))]
    use_graph = bool(case % 2)
    log(f"random batch case {case}: jobs={len(jobs)} pool={pool} chunk={chunk} graph={use_graph}")
    b = Batch(jobs)
    b.run(Batch.tuning(pool=pool, chunk_nodes=chunk, use_graph=use_graph))
    for j, (job, og) in enumerate(zip(jobs, graphs)):
        root = b.info[j]["root"]
        assert b.info[j]["n"] == og.n and root == (job["root"] if job["root"] >= 0 else csr.landmark(og))
        om, seed, sid, qid = job["omega"], job["seed"], job["stream_id"], job["qid"]
        r = b.result(j)
        w = native.wilson(og, root, om, seed, stream=sid, qid=qid)
        a1 = native.absorbed(og, root, om, seed, 1, stream=sid, qid=qid)
        a2 = native.absorbed(og, root, om, seed, 2, stream=sid, qid=qid, want_y2=False)
        assert np.array_equal(r["Y1"], w["Y1"][0]) and np.array_equal(r["y1"], w["y1"]), j
        assert np.array_equal(r["Y2"], a1["Y2"][0]) and np.array_equal(r["len_uniform"], a1["len"]), j
        assert np.array_equal(r["len_pi"], a2["len"]), j
    b.close()


def _spantree_oracle(og, root, omega, seed, B, begin, total, stream, qid):
    X1 = np.zeros((B, og.n), np.int64)
    X2 = np.zeros((B, og.n), np.int64)
    for b in range(B):
        lo = max(begin, -(-b * total // B))
        hi = min(begin + omega, -(-(b + 1) * total // B))
        if hi > lo:
            r = native.spantree(og, root, hi - lo, seed, 1, stream=stream, qid=qid, sample_begin=lo)
            X1[b], X2[b] = r["X1"], r["X2"]
    k = native.spantree(og, root, omega, seed, 2, stream=stream, qid=qid, sample_begin=begin)
    return dict(X1=X1, X2=X2, s1=k["s1"], s2=k["s2"])


@pytest.mark.parametrize("case", range(10))
def test_random_spantree_bit_exact(case):
    """SpanTree sums (lap_spantree) on random graphs, roots, sample ranges,
    block counts, seeds, stream and query ids, sampler forms and pools: the
    per-block X1, X2 and the per-sample s1, s2 equal the oracle's."""
    rng = np.random.default_rng(13100 + case)
    n, s, d, lcc = _graph(rng, case)
    og, hg = both(n, s, d, keep_lcc=lcc)
    root = int(rng.integers(0, og.n)) if case % 3 else csr.landmark(og)
    omega = int(rng.integers(1, 120))
    begin = int(rng.integers(0, 5))
    total = begin + omega + int(rng.integers(0, 5))
    B = int(rng.integers(1, min(total, 6) + 1))
    seed = int(rng.integers(1 << 62))
    stream = int(rng.integers(0, 4))
    qid = int(rng.integers(0, 1 << 40))
    mode, group = [(1, 0), (2, 0), (3, 2), (3, 4), (3, 8)][case % 5]
    pool = int(rng.integers(0, 40))
    log(f"random spantree case {case}: n={og.n} root={root} omega={omega} begin={begin} B={B} "
        f"mode={mode}/{group} pool={pool}")
    got = hg.spantree(omega, seed, root, B=B, sample_begin=begin, n_total=total, mode=mode, group=group, pool=pool,
                      stream_id=stream, qid=qid)
    exp = _spantree_oracle(og, root, omega, seed, B, begin, total, stream, qid)
    for k in ("X1", "X2", "s1", "s2"):
        assert np.array_equal(got[k], exp[k]), k


@pytest.mark.parametrize("case", range(10))
def test_random_loop_included_bit_exact(case):
    """Loop-included paths (lap_loop_included) on random graphs, roots, start
    kinds, sample ranges, block counts, seeds, ids, sampler forms and pools:
    departures per node and per path equal the oracle's."""
    rng = np.random.default_rng(15000 + case)
    n, s, d, lcc = _graph(rng, case)
    og, hg = both(n, s, d, keep_lcc=lcc)
    root = int(rng.integers(0, og.n)) if case % 3 else csr.landmark(og)
    tag = 1 + case % 2
    omega = int(rng.integers(1, 150))
    begin = int(rng.integers(0, 5))
    total = begin + omega + int(rng.integers(0, 5))
    B = int(rng.integers(1, min(total, 6) + 1))
    seed = int(rng.integers(1 << 62))
    stream = int(rng.integers(0, 4))
    qid = int(rng.integers(0, 1 << 40))
    mode, group = [(1, 0), (2, 0), (3, 2), (3, 4), (3, 8)][case % 5]
    pool = int(rng.integers(0, 40))
    log(f"random loops case {case}: n={og.n} root={root} tag={tag} omega={omega} begin={begin} B={B} "
        f"mode={mode}/{group} pool={pool}")
    got = hg.loop_included(omega, seed, tag, root, B=B, sample_begin=begin, n_total=total, mode=mode, group=group,
                           pool=pool, stream_id=stream, qid=qid)
    exp = native.loop_included(og, root, omega, seed, tag, stream=stream, qid=qid, sample_begin=begin,
                               omega_total=total, B=B)
    assert np.array_equal(got["Y2"], exp["Y2"]) and np.array_equal(got["len"], exp["len"])


@pytest.mark.parametrize("case", range(10))
def test_random_estimates_match_oracle_assembly(case):
    """FP64 estimates (lap_estimate, with the derived outputs) on random graphs,
    roots, sample counts, block counts, seeds, ids and sampler forms: every
    output equals the oracle's assembly of the oracle's counts to 1e-12
    (standard errors to 1e-9)."""
    from oracle import estimators
    rng = np.random.default_rng(17100 + case)
    n, s, d, lcc = _graph(rng, case)
    og, hg = both(n, s, d, keep_lcc=lcc)
    root = int(rng.integers(0, og.n)) if case % 3 else csr.landmark(og)
    omega = int(rng.integers(2, 300))
    B = int(rng.integers(1, min(omega, 8) + 1))
    seed = int(rng.integers(1 << 62))
    stream = int(rng.integers(0, 4))
    qid = int(rng.integers(0, 1 << 40))
    mode, group = [(1, 0), (2, 0), (3, 2), (3, 4), (3, 8)][case % 5]
    log(f"random estimate case {case}: n={og.n} root={root} omega={omega} B={B} mode={mode}/{group}")
    est = hg.estimate(omega, seed, root, B=B, lv=True, derived=True, mode=mode, group=group, stream_id=stream,
                      qid=qid)
    w = native.wilson(og, root, omega, seed, stream=stream, qid=qid, B=B)
    a = native.absorbed(og, root, omega, seed, 1, stream=stream, qid=qid, B=B)
    p = native.absorbed(og, root, omega, seed, 2, stream=stream, qid=qid, want_y2=False)
    diag, se = estimators.diag_ldagger_blocks(w["Y1"], a["Y2"], omega, og.deg)
    c, tr = estimators.closeness(diag)
    k, kse = estimators.kemeny(w["y1"], p["len"])
    np.testing.assert_allclose(est["diag"], diag, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(est["diag_se"], se, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(est["closeness"], c, rtol=1e-12)
    np.testing.assert_allclose(est["trace"][0], tr, rtol=1e-12)
    np.testing.assert_allclose(est["kemeny"][0], k, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(est["kemeny_se"][0], kse, rtol=1e-9, atol=1e-12)
    lv = w["Y1"].sum(0) / (omega * og.deg)
    lv[root] = 0.0
    np.testing.assert_allclose(est["lv_diag"], lv, rtol=1e-12)
    np.testing.assert_allclose(est["kirchhoff"][0], estimators.kirchhoff(diag), rtol=1e-12)
    np.testing.assert_allclose(est["rw_betweenness"], estimators.rw_betweenness(diag), rtol=1e-12)


@pytest.mark.parametrize("case", range(6))
def test_random_landmark_traces_bit_exact(case):
    """Landmark study (lap_landmark_traces) on random graphs with random root
    lists (repeats allowed) and sample counts: each root's mean draws equal
    the oracle's per-sample totals for that root exactly."""
    rng = np.random.default_rng(19000 + case)
    n, s, d, lcc = _graph(rng, case)
    og, hg = both(n, s, d, keep_lcc=lcc)
    roots = rng.integers(0, og.n, int(rng.integers(1, 40))).astype(np.int32)
    roots[0] = csr.landmark(og)
    omega = int(rng.integers(1, 100))
    seed = int(rng.integers(1 << 62))
    log(f"random landmark case {case}: n={og.n} roots={len(roots)} omega={omega}")
    tr, se = hg.landmark_traces(roots, omega, seed)
    for j, r in enumerate(roots):
        w = native.wilson(og, int(r), omega, seed, want_y1=False)
        assert tr[j] == int(w["y1"].sum()) / omega, (j, int(r))
