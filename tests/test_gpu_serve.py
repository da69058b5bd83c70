"""The serving loop: every query's result equals the oracle's (counts drawn
from the same keyed streams, FP64 assembly to 1e-12), a query's result is
identical alone and in a mix under different batching, Kemeny queries equal
the plain path with the same query id, and admission respects the result
arena."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr, estimators, native
from tests.gpu_common import both, er256_edges, log

pytestmark = pytest.mark.gpu

GLOBAL_QID = (1 << 64) - 1
SEED = 3


def _queries():
    return [dict(qid=1, kind=0, u=7, w=0, budget=200), dict(qid=2, kind=1, u=10, w=150, budget=300),
            dict(qid=3, kind=2, u=0, w=0, budget=48), dict(qid=4, kind=0, u=200, w=0, budget=1),
            dict(qid=5, kind=1, u=5, w=5, budget=64), dict(qid=6, kind=0, u=-1, w=0, budget=130),
            dict(qid=7, kind=2, u=0, w=0, budget=5), dict(qid=8, kind=1, u=-1, w=3, budget=65)]


def _setup():
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    qs = _queries()
    for q in qs:
        if q["u"] == -1:
            q["u"] = root                     # queries at the landmark itself
    return og, hg, root, qs


def _oracle_value(og, root, q, tr_lv, s_lv):
    b, qid = q["budget"], q["qid"]
    if q["kind"] == 0:
        r = native.query_walks(og, root, SEED, qid, q["u"], 0, q["u"], q["u"], b)
        c, _, _ = estimators.closeness_query(r["dep_a"], r["norm_len"], og.deg[q["u"]], og.n, tr_lv, s_lv)
        return c
    if q["kind"] == 1:
        fs = native.query_walks(og, root, SEED, qid, q["u"], 0, q["u"], q["w"], b)
        ft = native.query_walks(og, root, SEED, qid, q["w"], 1, q["w"], q["u"], b)
        r, _ = estimators.resistance_query(fs["dep_a"], fs["dep_b"], ft["dep_a"], ft["dep_b"],
                                           og.deg[q["u"]], og.deg[q["w"]])
        return r
    w = native.wilson(og, root, b, SEED, qid=qid)
    p = native.absorbed(og, root, b, SEED, 2, qid=qid, want_y2=False)
    k, _ = estimators.kemeny(w["y1"], p["len"])
    return k


def _run(hg, qs, **cfg):
    from paper_2311_10290_amd import Server
    srv = Server(hg, seed=SEED, global_samples=512, **cfg)
    for q in qs:
        srv.submit(q["qid"], q["kind"], q["budget"], q["u"], q["w"])
    res = srv.run_all(timeout_s=120)
    g = srv.globals()
    srv.close()
    assert len(res) == len(qs) and all(r["status"] == 0 for r in res)
    return {r["qid"]: r for r in res}, g


@pytest.mark.parametrize("wilson_group", [1, 8])
def test_server_matches_oracle(wilson_group):
    """wilson_group 1: Kemeny trees by single wavefronts; 8: by workgroups of 8."""
    og, hg, root, qs = _setup()
    log(f"serve: mixed run, wilson_group {wilson_group}")
    res, (tr_lv, s_lv) = _run(hg, qs, wilson_group=wilson_group)
    w = native.wilson(og, root, 512, SEED, qid=GLOBAL_QID)
    a = native.absorbed(og, root, 512, SEED, 1, qid=GLOBAL_QID)
    otr, os_ = estimators.globals_from_counts(w["Y1"][0], a["Y2"][0], 512, og.deg, root)
    np.testing.assert_allclose([tr_lv, s_lv], [otr, os_], rtol=1e-12)
    for q in qs:
        want = _oracle_value(og, root, q, tr_lv, s_lv)
        np.testing.assert_allclose(res[q["qid"]]["value"], want, rtol=1e-12, err_msg=str(q))


def test_alone_equals_mixed_under_any_batching():
    og, hg, root, qs = _setup()
    mixed, _ = _run(hg, qs)
    odd, _ = _run(hg, qs, launches=1, items_per_launch=3, waves=5)
    grouped, _ = _run(hg, qs, launches=4, items_per_launch=5, waves=3, wilson_group=4)
    for q in qs:
        alone, _ = _run(hg, [q], launches=3, items_per_launch=2, wilson_group=2)
        for other in (mixed, odd, grouped):
            assert alone[q["qid"]]["value"] == other[q["qid"]]["value"], q
            assert alone[q["qid"]]["se"] == other[q["qid"]]["se"] or np.isnan(alone[q["qid"]]["se"])


def test_kemeny_query_equals_plain_path():
    og, hg, root, qs = _setup()
    res, _ = _run(hg, [q for q in qs if q["kind"] == 2])
    for q in qs:
        if q["kind"] != 2:
            continue
        e = hg.estimate(q["budget"], SEED, root, B=1, se=False, diag=False, closeness=False, qid=q["qid"])
        assert e["kemeny"][0] == res[q["qid"]]["value"]


def test_admission_by_result_memory():
    from paper_2311_10290_amd import LapError, Server
    og, hg, root, _ = _setup()
    srv = Server(hg, seed=SEED, global_samples=64, arena_bytes=8 * 2 * 300, launches=2, items_per_launch=4)
    for i in range(12):
        srv.submit(100 + i, 0, 300, u=i * 7 % og.n)      # each needs the whole arena
    srv.step()
    p = srv.pending()
    assert p["active"] == 1 and p["queued"] == 11
    res = srv.run_all(timeout_s=120)
    assert sorted(r["qid"] for r in res) == list(range(100, 112))
    with pytest.raises(LapError):
        srv.submit(999, 0, 301, u=1)                      # can never fit
    srv.close()


def test_cancel_queued_and_running_queries():
    """Cancelling: a queued query leaves at once, a running one stops issuing
    work and gives its arena region back when its items on the device are
    done; both come back with status LAP_ECANCELED.  Every other query's
    result equals its result in a run without cancellations, and the whole
    arena is free again afterwards."""
    from paper_2311_10290_amd import LapError, Server
    og, hg, root, qs = _setup()
    ref, _ = _run(hg, qs)
    words = sum((4 if q["kind"] == 1 else 2) * q["budget"] for q in qs)
    srv = Server(hg, seed=SEED, global_samples=512, launches=2, items_per_launch=2, waves=3,
                 arena_bytes=8 * words, wilson_slots=2)
    for q in qs:
        srv.submit(q["qid"], q["kind"], q["budget"], q["u"], q["w"])
    srv.cancel(qs[-1]["qid"])                 # still queued
    srv.step()
    running = next(q for q in qs if q["budget"] > 100)
    srv.cancel(running["qid"])                # admitted, items on the device
    with pytest.raises(LapError) as ei:
        srv.cancel(123456789)
    assert ei.value.code == -1
    res = {r["qid"]: r for r in srv.run_all(timeout_s=120)}
    assert sorted(res) == sorted(q["qid"] for q in qs)
    for q in qs:
        r = res[q["qid"]]
        if q["qid"] in (qs[-1]["qid"], running["qid"]):
            assert r["status"] == -6 and np.isnan(r["value"]), q
        else:
            assert r["status"] == 0 and r["value"] == ref[q["qid"]]["value"], q
    assert srv.pending() == dict(queued=0, active=0, inflight=0)
    # the arena is whole again: one query as large as all of them together runs
    srv.submit(777, 0, words // 2, u=3)
    big = srv.run_all(timeout_s=120)
    assert len(big) == 1 and big[0]["status"] == 0
    srv.close()


def _random_graph(rng, case):
    kind = case % 3
    if kind == 0:
        n = int(rng.integers(40, 400))
        s, d = gg.erdos_renyi(n, float(rng.uniform(3.0, 8.0)) / n, int(rng.integers(1 << 30)))
    elif kind == 1:
        n = int(rng.integers(40, 2000))
        s, d = gg.barabasi_albert(n, int(rng.integers(1, 5)), int(rng.integers(1 << 30)))
    else:
        r, c = int(rng.integers(3, 25)), int(rng.integers(3, 25))
        n = r * c
        s, d = gg.grid(r, c)
    return n, s, d


@pytest.mark.parametrize("case", range(6))
def test_random_server_configs_match_oracle(case):
    """Random graphs, roots and query mixes under random server configurations:
    stream counts, slots per launch, items per launch, samples per Wilson item,
    Kemeny forms and result arenas small enough to hold back admission.  Every
    result and the cached global terms equal the oracle's."""
    from paper_2311_10290_amd import Server
    rng = np.random.default_rng(11000 + case)
    n, s, d = _random_graph(rng, case)
    og, hg = both(n, s, d, keep_lcc=True)
    root = csr.landmark(og) if case % 2 == 0 else int(rng.integers(0, og.n))
    qs, used = [], set()
    for _ in range(int(rng.integers(4, 21))):
        kind = int(rng.choice([0, 1, 2], p=[0.4, 0.4, 0.2]))
        qid = int(rng.integers(0, 1 << 40))
        while qid in used:
            qid = int(rng.integers(0, 1 << 40))
        used.add(qid)
        budget = int(rng.integers(1, 65 if kind == 2 else 301))
        u = root if rng.random() < 0.1 else int(rng.integers(0, og.n))
        w = int(rng.integers(0, og.n))
        qs.append(dict(qid=qid, kind=kind, u=u, w=w, budget=budget))
    words = max((4 if q["kind"] == 1 else 2) * q["budget"] for q in qs)
    cfg = dict(launches=int(rng.integers(1, 7)), waves=[0, 1, 3, 17, 64][int(rng.integers(0, 5))],
               items_per_launch=[0, 1, 2, 7, 50][int(rng.integers(0, 5))],
               wilson_chunk=[0, 1, 3][int(rng.integers(0, 3))], wilson_group=[0, 1, 2, 4, 8][int(rng.integers(0, 5))],
               arena_bytes=0 if rng.random() < 0.5 else 8 * words * int(rng.integers(1, 4)))
    cfg["wilson_slots"] = [0, 1, 2, 5][case % 4]
    G = int(rng.integers(16, 257))
    log(f"random serve case {case}: n={og.n} root={root} queries={len(qs)} cfg={cfg}")
    srv = Server(hg, seed=SEED, root=root, global_samples=G, **cfg)
    for q in qs:
        srv.submit(q["qid"], q["kind"], q["budget"], q["u"], q["w"])
    res = {r["qid"]: r for r in srv.run_all(timeout_s=120)}
    tr_lv, s_lv = srv.globals()
    srv.close()
    assert len(res) == len(qs) and all(r["status"] == 0 for r in res.values())
    w = native.wilson(og, root, G, SEED, qid=GLOBAL_QID)
    a = native.absorbed(og, root, G, SEED, 1, qid=GLOBAL_QID)
    otr, os_ = estimators.globals_from_counts(w["Y1"][0], a["Y2"][0], G, og.deg, root)
    np.testing.assert_allclose([tr_lv, s_lv], [otr, os_], rtol=1e-12)
    for q in qs:
        want = _oracle_value(og, root, q, tr_lv, s_lv)
        np.testing.assert_allclose(res[q["qid"]]["value"], want, rtol=1e-12, err_msg=str(q))
