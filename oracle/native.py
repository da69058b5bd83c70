"""ctypes binding of the oracle's C sampler (test infrastructure only).

Builds ``oracle/sampler.c`` with gcc into ``oracle/liboracle.so`` and wraps
its entry points.  See the header of ``sampler.c`` for the sampling rules.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

WILSON_TAG, UNIFORM_TAG, STATIONARY_TAG = 0, 1, 2


def build() -> str:
    src = os.path.join(_HERE, "sampler.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src])
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i64, i32, u64, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32
        P = ctypes.c_void_p
        L.oracle_philox4x64_10.argtypes = [P, P, P]
        L.oracle_philox4x64_10.restype = None
        L.oracle_map_below.argtypes = [u64, u64]
        L.oracle_map_below.restype = u64
        L.oracle_wilson.argtypes = [i64, P, P, i32, u64, u32, u64, i64, i64, i64, i32,
                                    P, P, P, i64, P, P, i32]
        L.oracle_wilson.restype = i32
        L.oracle_wilson_ordered.argtypes = [i64, P, P, i32, u64, u32, u64, i64, P, i64,
                                            P, P, P, i64, P]
        L.oracle_wilson_ordered.restype = i64
        L.oracle_wilson_scripted.argtypes = [i64, i32, P, P, P, i64, P, P, P, i64, P]
        L.oracle_wilson_scripted.restype = i64
        L.oracle_loop_included_path.argtypes = [i64, P, P, i32, u64, u32, u64, i64, P, P, i32,
                                                P, i64, P]
        L.oracle_loop_included_path.restype = i64
        L.oracle_absorbed.argtypes = [i64, P, P, i32, u64, u32, u64, i32, i64, i64, i64, i32,
                                      P, P, P, i64, P, i64, P, i32]
        L.oracle_absorbed.restype = i32
        L.oracle_query_walks.argtypes = [i64, P, P, i32, u64, u32, u64, i32, i32, i32, i32, i64, i64,
                                         P, P, P, P]
        L.oracle_query_walks.restype = i32
        L.oracle_loop_included.argtypes = [i64, P, P, i32, u64, u32, u64, i32, i64, i64, i64, i32, P, P, i32]
        L.oracle_loop_included.restype = i32
        L.oracle_pair_paths.argtypes = [i64, P, P, i32, u64, u32, u64, i64, i64, i64, i32, i64, P, P, P, i32]
        L.oracle_pair_paths.restype = i32
        L.oracle_lv_rows.argtypes = [i64, P, P, i32, u64, u32, u64, i64, i64, i64, i32, i64, P, P, i32]
        L.oracle_lv_rows.restype = i32
        L.oracle_bfs_tree.argtypes = [i64, P, P, i32, P]
        L.oracle_bfs_tree.restype = i64
        L.oracle_spantree_tree.argtypes = [i64, P, i32, P, P, P, P, P, P, P]
        L.oracle_spantree_tree.restype = None
        L.oracle_spantree.argtypes = [i64, P, P, i32, u64, u32, u64, i64, i64, i32, P, P, P, P, i32]
        L.oracle_spantree.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().oracle_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def map_below(x: int, d: int) -> int:
    return int(lib().oracle_map_below(x, d))


def _graph(g):
    return g.n, np.ascontiguousarray(g.rp, np.int64), np.ascontiguousarray(g.col, np.int32)


def wilson(g, root, omega, seed, *, stream=0, qid=0, sample_begin=0, n_samples=None, B=1,
           keep=(), want_y1=True, want_per_sample=True, threads=0):
    """Run Wilson samples [sample_begin, sample_begin+n_samples) of an omega-sample run.

    Returns dict with Y1 ([B, n] int64), y1 ([n_samples] int64) and, for the
    absolute sample indices in ``keep``, next/draws ([len(keep), n] int32).
    """
    n, rp, col = _graph(g)
    if n_samples is None:
        n_samples = omega - sample_begin
    Y1 = np.zeros((B, n), np.int64) if want_y1 else None
    y1 = np.zeros(n_samples, np.int64) if want_per_sample else None
    keep = np.ascontiguousarray(np.asarray(keep, np.int64))
    nk = len(keep)
    nxt = np.zeros((nk, n), np.int32)
    drw = np.zeros((nk, n), np.int32)
    st = lib().oracle_wilson(n, _p(rp), _p(col), int(root), seed, stream, qid, sample_begin,
                             n_samples, omega, B, _p(Y1), _p(y1), _p(keep), nk, _p(nxt), _p(drw),
                             threads)
    if st != 0:
        raise MemoryError("oracle_wilson failed")
    return dict(Y1=Y1, y1=y1, next=nxt, draws=drw)


def wilson_ordered(g, root, sample, seed, order, *, stream=0, qid=0, trace_cap=0):
    n, rp, col = _graph(g)
    order = np.ascontiguousarray(order, np.int32)
    nxt = np.zeros(n, np.int32)
    drw = np.zeros(n, np.int32)
    tr = np.zeros(max(trace_cap, 1), np.int32)
    tl = np.zeros(1, np.int64)
    tot = lib().oracle_wilson_ordered(n, _p(rp), _p(col), int(root), seed, stream, qid, sample,
                                      _p(order), len(order), _p(nxt), _p(drw),
                                      _p(tr) if trace_cap else None, trace_cap, _p(tl))
    return dict(total=int(tot), next=nxt, draws=drw, trace=tr[: int(tl[0])] if trace_cap else None)


def _stacks(stacks, n):
    vals, off = [], [0]
    for u in range(n):
        s = list(stacks.get(u, []))
        vals.extend(s)
        off.append(len(vals))
    return np.asarray(vals if vals else [0], np.int32), np.asarray(off, np.int64)


def wilson_scripted(n, root, stacks, order, trace_cap=256):
    """Wilson over explicit stacks {u: [S[u][0], S[u][1], ...]} (bottom first)."""
    sv, so = _stacks(stacks, n)
    order = np.ascontiguousarray(order, np.int32)
    nxt = np.zeros(n, np.int32)
    drw = np.zeros(n, np.int32)
    tr = np.zeros(trace_cap, np.int32)
    tl = np.zeros(1, np.int64)
    tot = lib().oracle_wilson_scripted(n, int(root), _p(sv), _p(so), _p(order), len(order),
                                       _p(nxt), _p(drw), _p(tr), trace_cap, _p(tl))
    if tot < 0:
        raise ValueError("scripted stack exhausted")
    return dict(total=int(tot), next=nxt, draws=drw, trace=tr[: int(tl[0])])


def loop_included_path(n, root, s, *, stacks=None, g=None, sample=0, seed=0, stream=0, qid=0,
                       trace_cap=1 << 16):
    if stacks is not None:
        sv, so = _stacks(stacks, n)
        rp = col = None
    else:
        sv = so = None
        _, rp, col = _graph(g)
    tr = np.zeros(trace_cap, np.int32)
    tl = np.zeros(1, np.int64)
    moves = lib().oracle_loop_included_path(n, _p(rp), _p(col), int(root), seed, stream, qid,
                                            sample, _p(sv), _p(so), int(s), _p(tr), trace_cap,
                                            _p(tl))
    if moves < 0:
        raise ValueError("loop-included path failed")
    return tr[: int(tl[0])]


def absorbed(g, root, n_walks, seed, tag, *, stream=0, qid=0, walk_begin=0, omega_total=None,
             B=1, want_y2=True, want_len=True, want_start=False, trace_walk=-1, trace_cap=0,
             threads=0):
    """v-absorbed walks: tag 1 uniform start (Alg. 2), tag 2 stationary start (Alg. 4)."""
    n, rp, col = _graph(g)
    if omega_total is None:
        omega_total = walk_begin + n_walks
    Y2 = np.zeros((B, n), np.int64) if want_y2 else None
    ln = np.zeros(n_walks, np.int64) if want_len else None
    sw = np.zeros(n_walks, np.int32) if want_start else None
    tr = np.zeros(max(trace_cap, 1), np.int32)
    tl = np.zeros(1, np.int64)
    lib().oracle_absorbed(n, _p(rp), _p(col), int(root), seed, stream, qid, tag, walk_begin,
                          n_walks, omega_total, B, _p(Y2), _p(ln), _p(sw), trace_walk,
                          _p(tr) if trace_cap else None, trace_cap, _p(tl), threads)
    return dict(Y2=Y2, len=ln, start=sw, trace=tr[: int(tl[0])] if trace_cap else None)


def query_walks(g, root, seed, qid, start, sub, a, b, n_walks, *, stream=0, walk_begin=0):
    """Walks from `start` absorbed at the root (sub-stream `sub`): departures
    from a and from b, normalised length, length, per walk."""
    n, rp, col = _graph(g)
    da = np.zeros(n_walks, np.int64)
    db = np.zeros(n_walks, np.int64)
    nl = np.zeros(n_walks)
    ln = np.zeros(n_walks, np.int64)
    lib().oracle_query_walks(n, _p(rp), _p(col), int(root), seed, stream, qid, int(start), int(sub), int(a),
                             int(b), walk_begin, n_walks, _p(da), _p(db), _p(nl), _p(ln))
    return dict(dep_a=da, dep_b=db, norm_len=nl, len=ln)


def bfs_tree(g, root):
    """BFS parent array from the root (neighbours in ascending order)."""
    n, rp, col = _graph(g)
    par = np.zeros(n, np.int32)
    reached = lib().oracle_bfs_tree(n, _p(rp), _p(col), int(root), _p(par))
    if reached != n:
        raise ValueError("graph not connected")
    return par


def spantree_tree(g, root, next_, weights=None, bfs_par=None):
    """Per-tree quantities of Alg. 1 / Alg. 3 for one spanning tree next_[]:
    path support ps, unit-flow voltage sums x1 and weighted-flow sums x2
    (weights default to 1: Alg. 1; degrees: Alg. 3)."""
    n = g.n
    nxt = np.ascontiguousarray(next_, np.int32)
    w = np.ones(n, np.int64) if weights is None else np.ascontiguousarray(weights, np.int64)
    par = bfs_tree(g, root) if bfs_par is None else np.ascontiguousarray(bfs_par, np.int32)
    ps = np.zeros(n, np.int64)
    x1 = np.zeros(n, np.int64)
    x2 = np.zeros(n, np.int64)
    scr = np.zeros(5 * n, np.int32)
    koff = np.zeros(n + 1, np.int64)
    lib().oracle_spantree_tree(n, _p(nxt), int(root), _p(par), _p(w), _p(ps), _p(x1), _p(x2), _p(scr), _p(koff))
    return dict(ps=ps, x1=x1, x2=x2, vis=scr[:n].copy(), fin=scr[n:2 * n].copy())


def spantree(g, root, n_samples, seed, kind, *, stream=0, qid=0, sample_begin=0, threads=0):
    """SpanTree sums over Wilson samples: kind 1 (Alg. 1) returns X1, X2 ([n]);
    kind 2 (Alg. 3) returns per-sample s1, s2 ([n_samples])."""
    n, rp, col = _graph(g)
    X1 = np.zeros(n, np.int64) if kind == 1 else None
    X2 = np.zeros(n, np.int64) if kind == 1 else None
    s1 = np.zeros(n_samples, np.int64) if kind == 2 else None
    s2 = np.zeros(n_samples, np.int64) if kind == 2 else None
    st = lib().oracle_spantree(n, _p(rp), _p(col), int(root), seed, stream, qid, sample_begin, n_samples, kind,
                               _p(X1), _p(X2), _p(s1), _p(s2), threads)
    if st != 0:
        raise RuntimeError(f"oracle_spantree failed ({st})")
    return dict(X1=X1, X2=X2, s1=s1, s2=s2)


def loop_included(g, root, n_paths, seed, tag, *, stream=0, qid=0, sample_begin=0, omega_total=None, B=1,
                  want_y2=True, threads=0):
    """Loop-included paths of Wilson samples, started like absorbed walks of
    kind tag: departures per node (Y2 [B][n]) and per path (len)."""
    n, rp, col = _graph(g)
    if omega_total is None:
        omega_total = sample_begin + n_paths
    Y2 = np.zeros((B, n), np.int64) if want_y2 else None
    ln = np.zeros(n_paths, np.int64)
    st = lib().oracle_loop_included(n, _p(rp), _p(col), int(root), seed, stream, qid, tag, sample_begin, n_paths,
                                    omega_total, B, _p(Y2), _p(ln), threads)
    if st != 0:
        raise MemoryError("oracle_loop_included failed")
    return dict(Y2=Y2, len=ln)


def pair_paths(g, root, n_samples, seed, s, t, *, stream=0, qid=0, sample_begin=0, omega_total=None, B=1,
               threads=0):
    """Loop-included paths from s_j and from t_j through the stacks of each
    Wilson sample: V [B][n_pairs][4] = departures (from s on the path from s,
    from t on the path from s, from t on the path from t, from s on the path
    from t)."""
    n, rp, col = _graph(g)
    if omega_total is None:
        omega_total = sample_begin + n_samples
    s = np.ascontiguousarray(s, np.int32)
    t = np.ascontiguousarray(t, np.int32)
    assert s.shape == t.shape
    V = np.zeros((B, len(s), 4), np.int64)
    st = lib().oracle_pair_paths(n, _p(rp), _p(col), int(root), seed, stream, qid, sample_begin, n_samples,
                                 omega_total, B, len(s), _p(s), _p(t), _p(V), threads)
    if st != 0:
        raise MemoryError("oracle_pair_paths failed")
    return V


def lv_rows(g, root, n_samples, seed, sources, *, stream=0, qid=0, sample_begin=0, omega_total=None, B=1,
            threads=0):
    """Loop-included paths from each source through the stacks of each Wilson
    sample: Y [B][n_sources][n] departures per node."""
    n, rp, col = _graph(g)
    if omega_total is None:
        omega_total = sample_begin + n_samples
    src = np.ascontiguousarray(sources, np.int32)
    Y = np.zeros((B, len(src), n), np.int64)
    st = lib().oracle_lv_rows(n, _p(rp), _p(col), int(root), seed, stream, qid, sample_begin, n_samples,
                              omega_total, B, len(src), _p(src), _p(Y), threads)
    if st != 0:
        raise MemoryError("oracle_lv_rows failed")
    return Y
