"""Parity at the full size of the mid workload (Barabasi-Albert n = 100,000,
m = 5, root = max degree, 2^12 samples) in the launch configuration the
benchmark uses: every integer count over all samples is compared with the
oracle (which runs the same samples on the host cores), plus per-node
next/draws of sampled trees."""
import numpy as np
import pytest

from oracle import csr, native
from tests.gpu_common import ba_edges, both, log

pytestmark = pytest.mark.gpu


def test_ba100k_counts_bit_exact():
    n, s, d = ba_edges(100_000, 5, 0)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega = 1 << 12
    keep = [0, 1, 2048, omega - 1]
    log("ba100k: HIP path")
    got = hg.sample_forests(omega, 1, root, y2=True, y2_pi=True, B=64, keep=keep)
    log("ba100k: oracle Wilson")
    w = native.wilson(og, root, omega, 1, B=64, keep=keep)
    assert np.array_equal(got["y1"], w["y1"])
    assert np.array_equal(got["Y1"], w["Y1"])
    assert np.array_equal(got["next"], w["next"]) and np.array_equal(got["draws"], w["draws"])
    log("ba100k: oracle absorbed walks")
    a = native.absorbed(og, root, omega, 1, 1, B=64)
    assert np.array_equal(got["Y2"], a["Y2"]) and np.array_equal(got["len_uniform"], a["len"])
    p = native.absorbed(og, root, omega, 1, 2, want_y2=False)
    assert np.array_equal(got["len_pi"], p["len"])


def test_rmat22_large_workload_counts_bit_exact():
    """The large workload at full size: R-MAT scale 22 (edge factor 16,
    a/b/c/d = .57/.19/.19/.05) largest component, root = max degree, 512
    samples, in the benchmark's launch configuration (automatic form: the
    workgroup sampler).  Every sample's total draws, the per-block counts and
    two sampled trees equal the oracle's."""
    import graphgen as gg
    from tests.gpu_common import both as _both
    s, d = gg.rmat(22, 16, seed=0)
    log("rmat22: CSR (both sides)")
    og, hg = _both(1 << 22, s, d, keep_lcc=True)
    del s, d
    root = csr.landmark(og)
    omega = 512
    keep = [0, omega - 1]
    log(f"rmat22 n={og.n}: HIP path")
    got = hg.sample_forests(omega, 1, root, B=64, keep=keep, y2=True, y2_pi=True)
    log("rmat22: oracle Wilson")
    w = native.wilson(og, root, omega, 1, B=64, keep=keep)
    assert np.array_equal(got["y1"], w["y1"])
    assert np.array_equal(got["Y1"], w["Y1"])
    assert np.array_equal(got["next"], w["next"]) and np.array_equal(got["draws"], w["draws"])
    # the absorbed walks of this graph step through arc records (large column array)
    log("rmat22: oracle absorbed walks")
    a = native.absorbed(og, root, omega, 1, 1, B=64)
    assert np.array_equal(got["Y2"], a["Y2"]) and np.array_equal(got["len_uniform"], a["len"])
    p = native.absorbed(og, root, omega, 1, 2, want_y2=False)
    assert np.array_equal(got["len_pi"], p["len"])


def test_batch512_workload_sampled_jobs_bit_exact():
    """The batching workload at full size: 512 graphs (ER with average degree
    in [8, 20] and BA with m in 2..8, n log-uniform in [1e3, 2e5], omega in
    [256, 4096], job-list seed 2) in one hipGraph-captured launch with the
    tuning the autotuner picks for it on the whole batch (6144 waves, chunks
    of 2^15 node-samples), as the benchmark runs it.  Four jobs -- the
    largest, the smallest and two more -- are compared with the oracle in
    every count, and in their FP64 estimates to 1e-12.  (Counts do not depend
    on the tuning; the randomised batch cases sweep pools and chunks.)"""
    import graphgen as gg
    from paper_2311_10290_amd import Batch
    from tests.test_gpu_batch import _check_job
    specs = gg.batch_jobs(512, seed=2)
    jobs = []
    for sp in specs:
        s, d = gg.job_edges(sp)
        jobs.append(dict(n=sp["n"], src=s, dst=d, keep_lcc=True, root=-1, omega=sp["omega"], seed=1,
                         stream_id=0, qid=0))
    log("batch512: full run, pool 6144, chunk 2^15, captured")
    b = Batch(jobs)
    b.run(Batch.tuning(pool=6144, chunk_nodes=1 << 15, use_graph=True))
    sizes = [j["n"] for j in jobs]
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 101, 358})
    for j in pick:
        log(f"batch512: job {j} n={jobs[j]['n']} omega={jobs[j]['omega']}")
        _check_job(b, jobs, j)
    assert b.stats()["trees"] == sum(j["omega"] for j in jobs)


def test_serving_rmat21_sampled_queries_match_oracle():
    """The serving workload at full size: R-MAT scale 21 largest component
    resident, default server configuration, a stream of mixed queries; a
    closeness, a resistance and a Kemeny query are recomputed by the oracle
    from the same keyed draws (values to 1e-12)."""
    import graphgen as gg
    from oracle import estimators
    from paper_2311_10290_amd import Server
    from tests.test_gpu_serve import GLOBAL_QID
    s, d = gg.rmat(21, 16, seed=0)
    og, hg = both(1 << 21, s, d, keep_lcc=True)
    del s, d
    root = csr.landmark(og)
    seed = 1
    log(f"rmat21 n={og.n}: server")
    srv = Server(hg, seed=seed, global_samples=256)
    qs = gg.query_stream(og.n, 60, qps=1.0, seed=3)
    for q in qs:
        srv.submit(q["qid"], q["kind"], q["budget"], q["u"], q["w"])
    res = {r["qid"]: r for r in srv.run_all(timeout_s=300)}
    tr_lv, s_lv = srv.globals()
    srv.close()
    assert len(res) == len(qs) and all(r["status"] == 0 for r in res.values())
    log("rmat21: oracle global terms")
    w = native.wilson(og, root, 256, seed, qid=GLOBAL_QID, want_per_sample=False)
    a = native.absorbed(og, root, 256, seed, 1, qid=GLOBAL_QID, want_len=False)
    otr, os_ = estimators.globals_from_counts(w["Y1"][0], a["Y2"][0], 256, og.deg, root)
    np.testing.assert_allclose([tr_lv, s_lv], [otr, os_], rtol=1e-12)
    done = set()
    for q in qs:
        if q["kind"] in done:
            continue
        done.add(q["kind"])
        b, qid = q["budget"], q["qid"]
        log(f"rmat21: oracle query kind {q['kind']} budget {b}")
        if q["kind"] == 0:
            r = native.query_walks(og, root, seed, qid, q["u"], 0, q["u"], q["u"], b)
            want, _, _ = estimators.closeness_query(r["dep_a"], r["norm_len"], og.deg[q["u"]], og.n, tr_lv, s_lv)
        elif q["kind"] == 1:
            fs = native.query_walks(og, root, seed, qid, q["u"], 0, q["u"], q["w"], b)
            ft = native.query_walks(og, root, seed, qid, q["w"], 1, q["w"], q["u"], b)
            want, _ = estimators.resistance_query(fs["dep_a"], fs["dep_b"], ft["dep_a"], ft["dep_b"],
                                                  og.deg[q["u"]], og.deg[q["w"]])
        else:
            ww = native.wilson(og, root, b, seed, qid=qid, want_y1=False)
            p = native.absorbed(og, root, b, seed, 2, qid=qid, want_y2=False)
            want, _ = estimators.kemeny(ww["y1"], p["len"])
        np.testing.assert_allclose(res[qid]["value"], want, rtol=1e-12, err_msg=str(q))
    assert done == {0, 1, 2}
