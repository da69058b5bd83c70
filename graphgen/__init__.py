"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module produces raw edge lists, fixed small graphs and workload
descriptions (job lists, query streams).  It contains none of the estimator
arithmetic: turning an edge list into a simple connected CSR graph, the
random walks and the estimators are implemented separately, once in the HIP
library and once in ``oracle/``.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build() -> str:
    """Compile gen.c into libgraphgen.so (gcc, -O2)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        p32 = ctypes.POINTER(ctypes.c_int32)
        lib.gg_erdos_renyi.argtypes = [i64, dbl, u64, i64, p32, p32]
        lib.gg_erdos_renyi.restype = i64
        lib.gg_barabasi_albert.argtypes = [i64, i64, u64, p32, p32]
        lib.gg_barabasi_albert.restype = i64
        lib.gg_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, p32, p32]
        lib.gg_rmat.restype = i64
        lib.gg_is_connected.argtypes = [i64, i64, p32, p32]
        lib.gg_is_connected.restype = i32
        lib.gg_hyperbolic.argtypes = [i64, dbl, dbl, u64, i64, p32, p32]
        lib.gg_hyperbolic.restype = i64
        lib.gg_hyperbolic_points.argtypes = [i64, dbl, dbl, u64, ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_hyperbolic_points.restype = dbl
        _lib = lib
    return _lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def erdos_renyi(n: int, p: float, seed: int):
    """G(n, p): each unordered pair present independently with probability p."""
    lib = _load()
    mean = p * n * (n - 1) / 2.0
    cap = int(mean + 10.0 * math.sqrt(max(mean, 1.0)) + 16)
    while True:
        src = np.empty(cap, np.int32)
        dst = np.empty(cap, np.int32)
        cnt = lib.gg_erdos_renyi(n, p, seed, cap, _p32(src), _p32(dst))
        if cnt <= cap:
            return src[:cnt].copy(), dst[:cnt].copy()
        cap = int(cnt)


def is_connected(n: int, src, dst) -> bool:
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    return bool(_load().gg_is_connected(n, len(src), _p32(src), _p32(dst)))


def erdos_renyi_connected(n: int, p: float, seed: int, max_attempts: int = 1000):
    """G(n, p) resampled until connected: attempt a uses seed*1_000_003 + a."""
    for a in range(max_attempts):
        src, dst = erdos_renyi(n, p, seed * 1_000_003 + a)
        if is_connected(n, src, dst):
            return src, dst, a
    raise RuntimeError("no connected G(n,p) sample within max_attempts")


def barabasi_albert(n: int, m: int, seed: int):
    """Preferential attachment from an (m+1)-node star; m edges per new node."""
    ne = m + (n - m - 1) * m
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    got = _load().gg_barabasi_albert(n, m, seed, _p32(src), _p32(dst))
    if got != ne:
        raise RuntimeError(f"gg_barabasi_albert failed ({got})")
    return src, dst


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 0):
    """Raw R-MAT pairs (self-loops and duplicates included)."""
    ne = edge_factor << scale
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    got = _load().gg_rmat(scale, edge_factor, a, b, c, seed, _p32(src), _p32(dst))
    if got != ne:
        raise RuntimeError(f"gg_rmat failed ({got})")
    return src, dst


def hyperbolic(n: int, avg_deg: float, gamma: float, seed: int):
    """Random hyperbolic graph (threshold model): power-law degrees with
    exponent gamma > 2 and average degree about avg_deg (raw pairs; may be
    disconnected)."""
    lib = _load()
    cap = int(n * avg_deg * 0.75 + 1024)
    while True:
        src = np.empty(cap, np.int32)
        dst = np.empty(cap, np.int32)
        cnt = lib.gg_hyperbolic(n, float(avg_deg), float(gamma), seed, cap, _p32(src), _p32(dst))
        if cnt < 0:
            raise ValueError("bad hyperbolic-graph arguments")
        if cnt <= cap:
            return src[:cnt].copy(), dst[:cnt].copy()
        cap = int(cnt)


def hyperbolic_points(n: int, avg_deg: float, gamma: float, seed: int):
    """(angles, radii, R) of the points hyperbolic() joins, for brute-force checks."""
    th = np.empty(n)
    r = np.empty(n)
    R = _load().gg_hyperbolic_points(n, float(avg_deg), float(gamma), seed, th.ctypes.data, r.ctypes.data)
    return th, r, R


# ---------------------------------------------------------------- small graphs
def _edges(pairs):
    a = np.asarray(pairs, np.int32).reshape(-1, 2)
    return a[:, 0].copy(), a[:, 1].copy()


def complete(n):
    return _edges([(i, j) for i in range(n) for j in range(i + 1, n)])


def cycle(n):
    return _edges([(i, (i + 1) % n) for i in range(n)])


def path(n):
    return _edges([(i, i + 1) for i in range(n - 1)])


def star(n):
    """Center 0, leaves 1..n-1."""
    return _edges([(0, i) for i in range(1, n)])


def diamond():
    """K4 minus the edge {2,3}: nodes 0,1 have degree 3, nodes 2,3 degree 2."""
    return _edges([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)])


def fig1_graph():
    """4-node graph whose stacks appear in the stack-representation figure:
    v1-v2, v1-v3, v2-v4, v3-v4 (ids 0..3 for v1..v4)."""
    return _edges([(0, 1), (0, 2), (1, 3), (2, 3)])


def grid(rows, cols):
    pairs = []
    for r in range(rows):
        for c in range(cols):
            u = r * cols + c
            if c + 1 < cols:
                pairs.append((u, u + 1))
            if r + 1 < rows:
                pairs.append((u, u + cols))
    return _edges(pairs)


# ------------------------------------------------------------- workload recipes
# The benchmark's workloads (graph recipe, preparation, landmark, sample
# budget, blocks, seeds) live in workloads.json beside this file.
_WORKLOADS = os.path.join(_HERE, "workloads.json")


def workload(name: str) -> dict:
    """Parameters of a benchmark workload: small, mid, large, batched, serving."""
    with open(_WORKLOADS) as f:
        table = json.load(f)
    if name not in table:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(table)}")
    return table[name]


def workload_edges(name: str):
    """(n, src, dst) of a graph workload, built from its recipe (before the
    largest-component and numbering steps, which the graph builder applies)."""
    g = workload(name)["graph"]
    fam = g["family"]
    if fam == "erdos_renyi_connected":
        s, d, _ = erdos_renyi_connected(g["n"], g["p"], g["seed"])
        return g["n"], s, d
    if fam == "barabasi_albert":
        s, d = barabasi_albert(g["n"], g["m"], g["seed"])
        return g["n"], s, d
    if fam == "rmat":
        s, d = rmat(g["scale"], g["edge_factor"], g["a"], g["b"], g["c"], seed=g["seed"])
        return 1 << g["scale"], s, d
    raise ValueError(f"unknown graph family {fam!r}")


def describe_workload(name: str) -> str:
    """One line naming a graph workload's recipe and parameters."""
    w = workload(name)
    g = w["graph"]
    fam = g["family"]
    if fam == "erdos_renyi_connected":
        text = f"ER({g['n']}, {g['p']}) seed {g['seed']} connected"
    elif fam == "barabasi_albert":
        text = f"Barabasi-Albert n={g['n']} m={g['m']}"
    else:
        d = round(1.0 - g["a"] - g["b"] - g["c"], 6)
        text = (f"R-MAT scale {g['scale']} (edge factor {g['edge_factor']}, a/b/c/d {g['a']}/{g['b']}/{g['c']}/{d}) "
                "symmetrised")
    if w.get("keep_lcc"):
        text += ", largest component"
    if w.get("degree_order"):
        text += " numbered by decreasing degree"
    if "omega" in w:
        text += f", root = max degree, omega = {w['omega']}, B = {w['blocks']}, Philox seed {w['philox_seed']}"
    return text


def batch_jobs(n_graphs: int = 512, seed: int = 2, n_lo: int = 1000, n_hi: int = 200_000,
               omega_lo: int = 256, omega_hi: int = 4096):
    """Job list for the many-graph batch: half ER (average degree uniform in
    [8, 20]), half BA (m uniform in {2..8}); n log-uniform in [n_lo, n_hi];
    sample budget uniform in [omega_lo, omega_hi]."""
    rng = np.random.default_rng(seed)
    jobs = []
    for g in range(n_graphs):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        omega = int(rng.integers(omega_lo, omega_hi + 1))
        if g % 2 == 0:
            davg = float(rng.uniform(8.0, 20.0))
            jobs.append(dict(kind="er", n=n, p=davg / (n - 1), davg=davg, omega=omega,
                             graph_seed=10_000 + g))
        else:
            m = int(rng.integers(2, 9))
            jobs.append(dict(kind="ba", n=n, m=m, omega=omega, graph_seed=10_000 + g))
    return jobs


def job_edges(job):
    if job["kind"] == "er":
        return erdos_renyi(job["n"], job["p"], job["graph_seed"])
    return barabasi_albert(job["n"], job["m"], job["graph_seed"])


def query_stream(n_nodes: int, n_queries: int, qps: float, seed: int = 3,
                 mix=(0.45, 0.45, 0.10), ecc_budget=(64, 1024), res_pairs: int = 1024,
                 kemeny_samples: int = 256):
    """Poisson arrivals at rate qps; query types 0 = single-node closeness
    (budget uniform in ecc_budget, log2-uniform), 1 = pairwise resistance
    (res_pairs walk pairs), 2 = Kemeny (kemeny_samples samples)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, n_queries)
    t = np.cumsum(gaps)
    kinds = rng.choice(3, size=n_queries, p=np.asarray(mix) / sum(mix))
    out = []
    lo, hi = math.log2(ecc_budget[0]), math.log2(ecc_budget[1])
    for q in range(n_queries):
        k = int(kinds[q])
        u = int(rng.integers(0, n_nodes))
        w = int(rng.integers(0, n_nodes))
        if k == 0:
            budget = int(round(2.0 ** rng.uniform(lo, hi)))
        elif k == 1:
            budget = res_pairs
        else:
            budget = kemeny_samples
        out.append(dict(qid=q, t=float(t[q]), kind=k, u=u, w=w, budget=budget))
    return out
