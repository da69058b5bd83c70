"""The oracle's sampler at the mid workload's full size (Barabasi-Albert
n = 100,000, m = 5, root = max degree), pinned by sparse solves instead of
dense inverses.  With N = (I - P_v)^{-1} = L_v^{-1} D_v (Lemma 1):

  E[draws of a Wilson sample at u]      = N_uu = d_u (L_v^{-1})_uu  (Lemma 4, Sec. 3.4)
  E[visits to u, uniform-start walk]    = (d_u / n) (L_v^{-1} 1)_u  (Lemma 5)
  E[length, uniform-start walk]         = 1^T L_v^{-1} d / n
  E[length, stationary-start walk]      = d^T L_v^{-1} d / 2m       (Sec. 5)

Every right-hand side is one conjugate-gradient solve with the SPD matrix
L_v.  Each mean is z-tested against its sampling error (batch means over 64
blocks for per-node counts, exact per-walk errors for lengths), Bonferroni
over the nodes tested."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import cg

import graphgen as gg
from oracle import csr, native

SEED = 7
OMEGA = 1024
B = 64
Z_MAX = 4.5       # 20 two-sided tests at 0.27% overall, t with 63 dof


@pytest.fixture(scope="module")
def ba100k():
    src, dst = gg.barabasi_albert(100_000, 5, 0)
    g = csr.build_csr(100_000, src, dst)
    v = csr.landmark(g)
    deg = np.diff(g.rp).astype(np.float64)
    rows = np.repeat(np.arange(g.n), np.diff(g.rp))
    A = sp.csr_matrix((np.ones(len(g.col)), (rows, g.col)), shape=(g.n, g.n))
    L = sp.diags(deg) - A
    keep = np.flatnonzero(np.arange(g.n) != v)
    Lv = L[keep][:, keep].tocsr()
    pick = np.random.default_rng(5).choice(keep, 16, replace=False)
    top = keep[np.argsort(-deg[keep], kind="stable")[:4]]
    nodes = np.concatenate([top, pick])
    return dict(g=g, v=v, deg=deg, Lv=Lv, keep=keep, nodes=nodes)


def _solve(Lv, b):
    x, info = cg(Lv, b, rtol=1e-12, maxiter=5000)
    assert info == 0
    return x


def _embed(f, x):
    out = np.zeros(f["g"].n)
    out[f["keep"]] = x
    return out


def _block_z(blocks, mean_exact):
    """z of the mean of B equal-weight block means against mean_exact."""
    m = blocks.mean(0)
    se = blocks.std(0, ddof=1) / np.sqrt(blocks.shape[0])
    return (m - mean_exact) / se


def test_wilson_draws_match_sparse_solves(ba100k):
    f = ba100k
    w = native.wilson(f["g"], f["v"], OMEGA, SEED, B=B, want_per_sample=False)
    per_block = w["Y1"][:, f["nodes"]] / (OMEGA / B)     # omega divisible by B: equal blocks
    exact = np.empty(len(f["nodes"]))
    pos = {u: i for i, u in enumerate(f["keep"])}
    for j, u in enumerate(f["nodes"]):
        e = np.zeros(len(f["keep"]))
        e[pos[u]] = 1.0
        exact[j] = f["deg"][u] * _solve(f["Lv"], e)[pos[u]]
    z = _block_z(per_block, exact)
    assert np.max(np.abs(z)) < Z_MAX, z


def test_uniform_walk_visits_and_length_match_sparse_solves(ba100k):
    f = ba100k
    g, n = f["g"], f["g"].n
    a = native.absorbed(g, f["v"], OMEGA, SEED, 1, B=B)
    x1 = _embed(f, _solve(f["Lv"], np.ones(len(f["keep"]))))
    exact = f["deg"][f["nodes"]] / n * x1[f["nodes"]]
    z = _block_z(a["Y2"][:, f["nodes"]] / (OMEGA / B), exact)
    assert np.max(np.abs(z)) < Z_MAX, z
    xd = _embed(f, _solve(f["Lv"], f["deg"][f["keep"]]))
    mean_len = xd.sum() / n
    ln = a["len"].astype(np.float64)
    zl = (ln.mean() - mean_len) / (ln.std(ddof=1) / np.sqrt(OMEGA))
    assert abs(zl) < 3.0, (ln.mean(), mean_len)
    # visits and length are two views of the same walks
    assert a["Y2"].sum() == a["len"].sum()


def test_stationary_walk_length_matches_sparse_solve(ba100k):
    f = ba100k
    g = f["g"]
    a = native.absorbed(g, f["v"], 4 * OMEGA, SEED, 2, want_y2=False)
    dk = f["deg"][f["keep"]]
    exact = dk @ _solve(f["Lv"], dk) / f["deg"].sum()
    ln = a["len"].astype(np.float64)
    z = (ln.mean() - exact) / (ln.std(ddof=1) / np.sqrt(len(ln)))
    assert abs(z) < 3.0, (ln.mean(), exact)
