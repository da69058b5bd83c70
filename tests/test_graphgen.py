"""Input generators are deterministic and produce the advertised shapes."""
import numpy as np
import pytest

import graphgen as gg


def test_er_deterministic_and_connected_resample():
    a = gg.erdos_renyi_connected(256, 0.05, 0)
    b = gg.erdos_renyi_connected(256, 0.05, 0)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all() and a[2] == b[2]
    assert gg.is_connected(256, a[0], a[1])
    assert ((a[0] >= 0) & (a[0] < a[1]) & (a[1] < 256)).all()


def test_er_density():
    s, d = gg.erdos_renyi(2000, 0.01, 5)
    exp = 0.01 * 2000 * 1999 / 2
    assert abs(len(s) - exp) < 6 * np.sqrt(exp)
    key = s.astype(np.int64) * 2000 + d
    assert len(np.unique(key)) == len(key)


def test_ba_shape():
    s, d = gg.barabasi_albert(1000, 3, 1)
    assert len(s) == 3 + (1000 - 4) * 3
    assert (s != d).all()
    deg = np.bincount(np.concatenate([s, d]), minlength=1000)
    assert deg.min() >= 1 and deg.max() > 30


def test_rmat_shape():
    s, d = gg.rmat(10, 8, seed=3)
    assert len(s) == 8 << 10
    assert s.max() < 1024 and d.max() < 1024
    # quadrant a = 0.57 dominates: many edges with both top bits clear
    assert ((s < 512) & (d < 512)).mean() > 0.5


def test_batch_and_query_recipes():
    jobs = gg.batch_jobs(512)
    assert len(jobs) == 512
    ns = np.array([j["n"] for j in jobs])
    om = np.array([j["omega"] for j in jobs])
    assert ns.min() >= 1000 and ns.max() <= 200_000 and om.min() >= 256 and om.max() <= 4096
    q = gg.query_stream(1000, 500, 100.0)
    assert len(q) == 500 and all(q[i]["t"] < q[i + 1]["t"] for i in range(499))


@pytest.mark.parametrize("gamma", [2.2, 2.6, 3.0])
def test_hyperbolic_pairs_equal_brute_force(gamma):
    """The band search emits exactly the pairs within hyperbolic distance R."""
    n = 1500
    s, d = gg.hyperbolic(n, 8.0, gamma, 11)
    th, r, R = gg.hyperbolic_points(n, 8.0, gamma, 11)
    ch = (np.cosh(r)[:, None] * np.cosh(r)[None, :]
          - np.sinh(r)[:, None] * np.sinh(r)[None, :] * np.cos(th[:, None] - th[None, :]))
    close = ch <= np.cosh(R)
    np.fill_diagonal(close, False)
    want = {(int(a), int(b)) for a, b in zip(*np.nonzero(np.triu(close)))}
    got = {(min(int(a), int(b)), max(int(a), int(b))) for a, b in zip(s, d)}
    assert len(got) == len(s)                       # every pair once
    # pairs at distance within rounding of R may go either way; all others agree
    tie = np.abs(ch - np.cosh(R)) <= 1e-9 * np.cosh(R)
    diff = got ^ want
    assert all(tie[a, b] for a, b in diff), len(diff)


def test_hyperbolic_degree_tail():
    """Average degree near the target and a heavier tail for smaller gamma."""
    n = 100_000
    tails = []
    for gamma in (2.5, 3.0):
        s, d = gg.hyperbolic(n, 10.0, gamma, 3)
        deg = np.bincount(np.concatenate([s, d]), minlength=n)
        assert 7.0 < deg.mean() < 13.0
        tails.append(np.sort(deg)[-n // 1000:].mean())
    assert tails[0] > 1.5 * tails[1]


def test_workload_table():
    """Every benchmark workload is in the table; the graph recipes build the
    edge lists the generators give for the same parameters, and the
    descriptions name them."""
    for name in ("small", "mid", "large", "batched", "serving"):
        w = gg.workload(name)
        assert w.get("philox_seed", 1) == 1
    with pytest.raises(KeyError):
        gg.workload("no such workload")
    n, s, d = gg.workload_edges("small")
    s2, d2, _ = gg.erdos_renyi_connected(256, 0.05, 0)
    assert n == 256 and np.array_equal(s, s2) and np.array_equal(d, d2)
    n, s, d = gg.workload_edges("mid")
    s2, d2 = gg.barabasi_albert(100_000, 5, 0)
    assert n == 100_000 and np.array_equal(s, s2) and np.array_equal(d, d2)
    assert gg.workload("large")["graph"]["scale"] == 22 and gg.workload("serving")["graph"]["scale"] == 21
    assert "ER(256, 0.05)" in gg.describe_workload("small")
    assert "Barabasi-Albert n=100000 m=5" in gg.describe_workload("mid")
    text = gg.describe_workload("large")
    assert "R-MAT scale 22" in text and "0.57/0.19/0.19/0.05" in text and "largest component" in text
    b = gg.workload("batched")
    jobs = gg.batch_jobs(b["jobs"], seed=b["job_seed"], n_lo=b["n_range"][0], n_hi=b["n_range"][1],
                         omega_lo=b["omega_range"][0], omega_hi=b["omega_range"][1])
    assert jobs == gg.batch_jobs(512)
    sv = gg.workload("serving")
    assert len(sv["loads"]) == len(sv["load_stream_seeds"]) and abs(sum(sv["mix"]) - 1.0) < 1e-12
