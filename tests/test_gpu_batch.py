"""The batched persistent launch: every job's counts equal the oracle's (and
the plain path's) bit for bit, estimates match the oracle assembly, and a
captured hipGraph replays correctly several times with eager work between
replays."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr, estimators, native
from tests.gpu_common import log

pytestmark = pytest.mark.gpu


def _jobs():
    jobs = []
    specs = [("er", 300, 0.04, 300, -1), ("ba", 500, 2, 257, -1), ("ba", 2000, 3, 64, 5), ("er", 1000, 0.012, 130, -1),
             ("ba", 120, 4, 1000, 7), ("er", 80, 0.1, 33, 0), ("ba", 5000, 2, 100, -1), ("er", 2500, 0.004, 200, -1)]
    for i, (kind, n, p, omega, root) in enumerate(specs):
        if kind == "er":
            s, d = gg.erdos_renyi(n, p, 100 + i)
        else:
            s, d = gg.barabasi_albert(n, p, 100 + i)
        jobs.append(dict(n=n, src=s, dst=d, keep_lcc=True, root=root, omega=omega, seed=1 + i % 3,
                         stream_id=i % 2, qid=0))
    return jobs


def _check_job(b, jobs, j):
    job = jobs[j]
    og = csr.build_csr(job["n"], job["src"], job["dst"], keep_lcc=True)
    inf = b.info[j]
    root = inf["root"]
    assert inf["n"] == og.n and (job["root"] >= 0 or root == csr.landmark(og))
    om, seed, sid = job["omega"], job["seed"], job["stream_id"]
    r = b.result(j)
    w = native.wilson(og, root, om, seed, stream=sid)
    a1 = native.absorbed(og, root, om, seed, 1, stream=sid)
    a2 = native.absorbed(og, root, om, seed, 2, stream=sid, want_y2=False)
    assert np.array_equal(r["Y1"], w["Y1"][0]) and np.array_equal(r["y1"], w["y1"])
    assert np.array_equal(r["Y2"], a1["Y2"][0]) and np.array_equal(r["len_uniform"], a1["len"])
    assert np.array_equal(r["len_pi"], a2["len"])
    diag = estimators.diag_ldagger(w["Y1"][0], a1["Y2"][0], om, og.deg)
    c, tr = estimators.closeness(diag)
    k, kse = estimators.kemeny(w["y1"], a2["len"])
    np.testing.assert_allclose(r["diag"], diag, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["closeness"], c, rtol=1e-12)
    np.testing.assert_allclose(r["trace"][0], tr, rtol=1e-12)
    np.testing.assert_allclose(r["kemeny"][0], k, rtol=1e-12)
    np.testing.assert_allclose(r["kemeny_se"][0], kse, rtol=1e-9)
    return r


def test_batch_bit_exact_eager():
    from paper_2311_10290_amd import Batch
    jobs = _jobs()
    b = Batch(jobs)
    for pool, chunk in [(0, 0), (5, 1000), (200, 1 << 20)]:
        log(f"batch eager pool {pool} chunk {chunk}")
        b.run(Batch.tuning(pool=pool, chunk_nodes=chunk, use_graph=False))
        for j in range(len(jobs)):
            _check_job(b, jobs, j)
        st = b.stats()
        assert st["trees"] == sum(j["omega"] for j in jobs)


def test_batch_with_degenerate_jobs():
    """A single-node graph (no edges: every count and estimate is zero), a
    single edge, a star with one sample and two ordinary jobs share one
    launch, eagerly and from the captured graph."""
    from paper_2311_10290_amd import Batch
    s5, d5 = gg.barabasi_albert(700, 3, 41)
    s6, d6 = gg.erdos_renyi(400, 0.03, 42)
    star = np.arange(1, 40, dtype=np.int32)
    jobs = [dict(n=1, src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32), keep_lcc=True, root=-1, omega=5, seed=2,
                 stream_id=0, qid=0),
            dict(n=2, src=np.array([0], np.int32), dst=np.array([1], np.int32), keep_lcc=True, root=-1, omega=7,
                 seed=3, stream_id=1, qid=0),
            dict(n=700, src=s5, dst=d5, keep_lcc=True, root=-1, omega=129, seed=1, stream_id=0, qid=0),
            dict(n=40, src=np.zeros(39, np.int32), dst=star, keep_lcc=True, root=5, omega=1, seed=4, stream_id=0,
                 qid=0),
            dict(n=400, src=s6, dst=d6, keep_lcc=True, root=-1, omega=64, seed=2, stream_id=1, qid=0)]
    b = Batch(jobs)
    for use_graph in (False, True):
        log(f"batch with degenerate jobs, graph {use_graph}")
        b.run(Batch.tuning(pool=3, chunk_nodes=256, use_graph=use_graph))
        r = b.result(0)
        assert b.info[0]["n"] == 1
        for k in ("Y1", "Y2", "y1", "len_uniform", "len_pi", "diag", "closeness", "trace", "kemeny"):
            assert not np.any(r[k]), k
        for j in range(1, len(jobs)):
            _check_job(b, jobs, j)
        assert b.stats()["trees"] == sum(j["omega"] for j in jobs)


def test_batch_equals_plain_path():
    from paper_2311_10290_amd import Batch, Graph
    jobs = _jobs()[:3]
    b = Batch(jobs)
    b.run(Batch.tuning(use_graph=False))
    for j, job in enumerate(jobs):
        g = Graph(job["n"], job["src"], job["dst"], keep_lcc=True)
        got = g.sample_forests(job["omega"], job["seed"], b.info[j]["root"], y2=True, y2_pi=True,
                               stream_id=job["stream_id"])
        r = b.result(j)
        assert np.array_equal(r["Y1"], got["Y1"][0]) and np.array_equal(r["y1"], got["y1"])
        assert np.array_equal(r["Y2"], got["Y2"][0]) and np.array_equal(r["len_pi"], got["len_pi"])


def test_batch_graph_replays():
    from paper_2311_10290_amd import Batch, Graph
    jobs = _jobs()
    b = Batch(jobs)
    b.run(Batch.tuning(use_graph=False))
    ref = [b.result(j) for j in range(len(jobs))]
    side = Graph(jobs[0]["n"], jobs[0]["src"], jobs[0]["dst"], keep_lcc=True)
    for rep in range(3):
        log(f"graph replay {rep}")
        b.run(Batch.tuning(use_graph=True))
        side.estimate(64, 9, B=4)                      # eager work between replays
        for j in range(len(jobs)):
            r = b.result(j)
            for k in ("Y1", "Y2", "y1", "len_uniform", "len_pi", "diag", "closeness", "kemeny"):
                assert np.array_equal(r[k], ref[j][k]), (rep, j, k)


def test_batch_graph_recaptured_after_item_table_moves():
    """A captured launch bakes in the item table's address and length.  An
    eager run at a smaller chunk size grows (and so moves) the table; the
    next captured run at the first chunk size must capture again instead of
    replaying the old launch.  Every job equals the eager run bit for bit."""
    from paper_2311_10290_amd import Batch
    jobs = _jobs()
    b = Batch(jobs)
    keys = ("Y1", "Y2", "y1", "len_uniform", "len_pi", "diag", "closeness", "kemeny", "kemeny_se")
    log("graph run, chunk 2^17")
    b.run(Batch.tuning(chunk_nodes=1 << 17, use_graph=True))
    first = [b.result(j) for j in range(len(jobs))]
    log("eager run, chunk 2^15")
    b.run(Batch.tuning(chunk_nodes=1 << 15, use_graph=False))
    ref = [b.result(j) for j in range(len(jobs))]
    log("graph run, chunk 2^17 again")
    b.run(Batch.tuning(chunk_nodes=1 << 17, use_graph=True))
    for j in range(len(jobs)):
        r = b.result(j)
        for k in keys:
            assert np.array_equal(r[k], ref[j][k]), (j, k)
            assert np.array_equal(first[j][k], ref[j][k]), (j, k)


def test_batch_autotune_returns_a_working_tuning():
    from paper_2311_10290_amd import Batch
    jobs = _jobs()[:4]
    b = Batch(jobs)
    t, ms = b.autotune()
    assert ms > 0 and t.pool > 0 and t.chunk_nodes > 0 and t.use_graph == 1
    b.run(t)
    for j in range(len(jobs)):
        _check_job(b, jobs, j)


def test_landmark_traces_match_oracle_and_dense():
    """Landmark study: per-root mean Wilson draws equal the oracle's per-sample
    totals (bit-exact) and agree with Tr((I-P_v)^{-1}) from a dense solve."""
    import math
    from oracle import dense
    from tests.gpu_common import both, er256_edges
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    roots = [0, 5, 100, csr.landmark(og), 255]
    omega = 600
    tr, se = hg.landmark_traces(roots, omega, 13)
    L = dense.laplacian(og)
    for j, r in enumerate(roots):
        w = native.wilson(og, r, omega, 13, want_y1=False)
        assert tr[j] == int(w["y1"].sum()) / omega
        exact = float(np.trace(dense.walk_green(L, r)))
        assert abs(tr[j] - exact) < 4.5 * se[j]
