"""Input generators are deterministic and produce the advertised shapes."""
import numpy as np

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
