"""Python binding of liblap (argument marshalling only).

Graph(n, src, dst)            -> lap_build_csr
Graph.sample_forests(...)     -> lap_sample_forests   (integer counts)
Graph.estimate(...)           -> lap_estimate         (diag(L^dagger), closeness, Kemeny)
diag_Ldagger / ecc / kemeny   -> the convenience entry points
Outputs are numpy arrays, or caller-supplied torch device tensors when
``device_out=True``.  ``stream`` is a raw hipStream_t (int) or a torch stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _capi as C


class LapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lap status {code}: {msg}")
        self.code = code


_lib = None


def load_library():
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime.  Loaded first, it also serves
        # liblap (same soname), so torch's streams and device tensors are
        # valid in the library's calls; loaded after liblap, a second runtime
        # would come up beside the first and could not see the device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(C.LIB_PATH):
            raise ImportError(f"{C.LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_2311_10290_amd/build.py")
        _lib = C.declare(ctypes.CDLL(C.LIB_PATH))
    return _lib


def _default_timeout():
    # kernel time limit in seconds (0 = the library default)
    return float(os.environ.get("LAP_TIMEOUT_S", "0") or 0)


def _check(rc):
    if rc != C.LAP_OK:
        raise LapError(rc, load_library().lap_last_error().decode())


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())      # torch tensor


def prof_enable(on=True):
    _check(load_library().lap_prof_enable(1 if on else 0))


def prof_reset():
    _check(load_library().lap_prof_reset())


def prof_read(kernel):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(load_library().lap_prof_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


class Graph:
    """A prepared graph resident on the current HIP device (lap_build_csr)."""

    def __init__(self, n, src, dst, keep_lcc=False, degree_order=False, stream=None):
        lib = load_library()
        src = np.ascontiguousarray(src, np.int32)
        dst = np.ascontiguousarray(dst, np.int32)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        h = ctypes.c_void_p()
        flags = (C.LAP_KEEP_LCC if keep_lcc else 0) | (C.LAP_DEGREE_ORDER if degree_order else 0)
        _check(lib.lap_build_csr(int(n), len(src), _ptr(src), _ptr(dst), flags, _stream(stream), ctypes.byref(h)))
        self._h = h
        n_ = ctypes.c_int64()
        nnz = ctypes.c_int64()
        mdn = ctypes.c_int32()
        md = ctypes.c_int32()
        _check(lib.lap_graph_info(h, ctypes.byref(n_), ctypes.byref(nnz), ctypes.byref(mdn), ctypes.byref(md)))
        self.n, self.nnz, self.max_deg_node, self.max_deg = n_.value, nnz.value, mdn.value, md.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().lap_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def csr(self):
        rp = np.zeros(self.n + 1, np.int64)
        col = np.zeros(self.nnz, np.int32)
        old = np.zeros(self.n, np.int32)
        _check(load_library().lap_graph_copy_csr(self._h, _ptr(rp), _ptr(col), _ptr(old)))
        return rp, col, old

    def _args(self, omega, seed, root, want, B, sample_begin, n_total, mode, pool, stream_id, qid, timeout_s,
              schedule=0, group=0, walks=0):
        return C.SampleArgs(n_samples=int(omega), seed=int(seed), root=int(root), stream=int(stream_id),
                            qid=int(qid), want=int(want), n_blocks=int(B), sample_begin=int(sample_begin),
                            n_total=int(n_total), mode=int(mode), pool=int(pool),
                            timeout_s=float(timeout_s) if timeout_s else _default_timeout(),
                            schedule=int(schedule), group=int(group), walks=int(walks))

    def sample_forests(self, omega, seed, root=-1, *, y1=True, y2=False, y2_pi=False, per_sample=True,
                       B=1, keep=(), sample_begin=0, n_total=0, mode=0, pool=0, stream_id=0, qid=0,
                       timeout_s=0.0, schedule=0, group=0, stream=None):
        """Integer counts of lap_sample_forests as numpy arrays."""
        n = self.n
        want = ((C.LAP_WANT_Y1 if y1 else 0) | (C.LAP_WANT_Y2_UNIFORM if y2 else 0)
                | (C.LAP_WANT_Y2_PI if y2_pi else 0) | (C.LAP_WANT_PER_SAMPLE if per_sample else 0))
        a = self._args(omega, seed, root, want, B, sample_begin, n_total, mode, pool, stream_id, qid, timeout_s,
                       schedule, group)
        keep = np.ascontiguousarray(np.asarray(list(keep), np.int64))
        nk = len(keep)
        out = dict(
            Y1=np.zeros((B, n), np.int64) if y1 else None,
            Y2=np.zeros((B, n), np.int64) if y2 else None,
            y1=np.zeros(omega, np.int64) if per_sample else None,
            len_uniform=np.zeros(omega, np.int64) if y2 else None,
            len_pi=np.zeros(omega, np.int64) if y2_pi else None,
            next=np.zeros((nk, n), np.int32) if nk else None,
            draws=np.zeros((nk, n), np.int32) if nk else None,
        )
        c = C.Counts(y1=_ptr(out["Y1"]), y2=_ptr(out["Y2"]), y1_per_sample=_ptr(out["y1"]),
                     y2len_uniform=_ptr(out["len_uniform"]), y2len_pi=_ptr(out["len_pi"]),
                     keep_idx=_ptr(keep) if nk else None, n_keep=nk,
                     next=_ptr(out["next"]), draws=_ptr(out["draws"]))
        _check(load_library().lap_sample_forests(self._h, ctypes.byref(a), ctypes.byref(c), _stream(stream)))
        return out

    def sample_forests_noalloc(self, omega, seed, root=-1, *, y1=True, y2=False, y2_pi=False, per_sample=True,
                               B=1, keep=(), sample_begin=0, n_total=0, mode=0, pool=0, stream_id=0, qid=0,
                               timeout_s=0.0, schedule=0, group=0, stream=None, out=None):
        """lap_sample_forests_noalloc: the same counts as sample_forests, written
        into caller-owned torch device tensors (``out``: Y1, Y2 [B, n], y1,
        len_uniform, len_pi [omega], next, draws [len(keep), n]; int64 except
        next/draws int32).  Without ``out`` the tensors are made here, before
        the call.  Returns the dict of tensors."""
        import torch
        n = self.n
        keep = np.ascontiguousarray(np.asarray(list(keep), np.int64))
        nk = len(keep)
        if out is None:
            dev = torch.device("cuda", torch.cuda.current_device())
            z = lambda *shape, dt=torch.int64: torch.zeros(*shape, dtype=dt, device=dev)
            out = dict(Y1=z(B, n) if y1 else None, Y2=z(B, n) if y2 else None,
                       y1=z(omega) if per_sample else None, len_uniform=z(omega) if y2 else None,
                       len_pi=z(omega) if y2_pi else None,
                       next=z(nk, n, dt=torch.int32) if nk else None, draws=z(nk, n, dt=torch.int32) if nk else None)
        want = ((C.LAP_WANT_Y1 if y1 else 0) | (C.LAP_WANT_Y2_UNIFORM if y2 else 0)
                | (C.LAP_WANT_Y2_PI if y2_pi else 0) | (C.LAP_WANT_PER_SAMPLE if per_sample else 0)
                | C.LAP_OUT_DEVICE)
        a = self._args(omega, seed, root, want, B, sample_begin, n_total, mode, pool, stream_id, qid, timeout_s,
                       schedule, group)
        c = C.Counts(y1=_ptr(out.get("Y1")), y2=_ptr(out.get("Y2")), y1_per_sample=_ptr(out.get("y1")),
                     y2len_uniform=_ptr(out.get("len_uniform")), y2len_pi=_ptr(out.get("len_pi")),
                     keep_idx=_ptr(keep) if nk else None, n_keep=nk,
                     next=_ptr(out.get("next")), draws=_ptr(out.get("draws")))
        _check(load_library().lap_sample_forests_noalloc(self._h, ctypes.byref(a), ctypes.byref(c), _stream(stream)))
        return out

    def estimate(self, omega, seed, root=-1, *, diag=True, se=True, lv=False, closeness=True, kemeny=True,
                 derived=False, B=64, mode=0, pool=0, stream_id=0, qid=0, timeout_s=0.0, group=0, stream=None,
                 out=None, walks=0):
        """FP64 estimates of lap_estimate.  With ``out`` (a dict of torch device
        tensors: diag, diag_se, lv_diag, closeness [n]; trace, kemeny,
        kemeny_se [1]) results are written there on the device."""
        n = self.n
        dev = out is not None
        want = C.LAP_OUT_DEVICE if dev else 0
        a = self._args(omega, seed, root, want, B if se else 1, 0, 0, mode, pool, stream_id, qid, timeout_s,
                       group=group, walks=walks)
        if dev:
            res = out
        else:
            res = dict(
                diag=np.zeros(n) if diag else None, diag_se=np.zeros(n) if (diag and se) else None,
                lv_diag=np.zeros(n) if lv else None, closeness=np.zeros(n) if closeness else None,
                trace=np.zeros(1) if (diag or closeness) else None, kemeny=np.zeros(1) if kemeny else None,
                kemeny_se=np.zeros(1) if kemeny else None, kirchhoff=np.zeros(1) if derived else None,
                rw_betweenness=np.zeros(n) if derived else None)
        e = C.Estimates(**{k: _ptr(res.get(k)) for k in
                           ("diag", "diag_se", "lv_diag", "closeness", "trace", "kemeny", "kemeny_se", "kirchhoff",
                            "rw_betweenness")})
        _check(load_library().lap_estimate(self._h, ctypes.byref(a), ctypes.byref(e), _stream(stream)))
        return res

    def spantree(self, omega, seed, root=-1, *, B=1, sample_begin=0, n_total=0, mode=0, pool=0, group=0,
                 stream_id=0, qid=0, timeout_s=0.0, schedule=0, stream=None):
        """SpanTree per-tree sums (lap_spantree): X1, X2 [B][n]; s1, s2 [omega]."""
        a = self._args(omega, seed, root, 0, B, sample_begin, n_total, mode, pool, stream_id, qid, timeout_s,
                       schedule, group)
        out = dict(X1=np.zeros((B, self.n), np.int64), X2=np.zeros((B, self.n), np.int64),
                   s1=np.zeros(omega, np.int64), s2=np.zeros(omega, np.int64))
        _check(load_library().lap_spantree(self._h, ctypes.byref(a), _ptr(out["X1"]), _ptr(out["X2"]),
                                           _ptr(out["s1"]), _ptr(out["s2"]), _stream(stream)))
        return out

    def spantree_estimate(self, omega, seed, root=-1, *, B=64, mode=0, pool=0, group=0, stream_id=0, qid=0,
                          timeout_s=0.0, stream=None):
        """SpanTree FP64 estimates (lap_spantree_estimate)."""
        a = self._args(omega, seed, root, 0, B, 0, 0, mode, pool, stream_id, qid, timeout_s, group=group)
        res = dict(diag=np.zeros(self.n), diag_se=np.zeros(self.n), closeness=np.zeros(self.n),
                   kemeny=np.zeros(1), kemeny_se=np.zeros(1))
        _check(load_library().lap_spantree_estimate(self._h, ctypes.byref(a), *[_ptr(res[k]) for k in
                                                    ("diag", "diag_se", "closeness", "kemeny", "kemeny_se")],
                                                    _stream(stream)))
        return res

    def loop_included(self, omega, seed, tag, root=-1, *, B=1, sample_begin=0, n_total=0, mode=0, pool=0, group=0,
                      stream_id=0, qid=0, timeout_s=0.0, stream=None):
        """Loop-included paths of the Wilson stacks (lap_loop_included): Y2 [B][n], len [omega]."""
        a = self._args(omega, seed, root, 0, B, sample_begin, n_total, mode, pool, stream_id, qid, timeout_s,
                       group=group)
        out = dict(Y2=np.zeros((B, self.n), np.int64), len=np.zeros(omega, np.int64))
        _check(load_library().lap_loop_included(self._h, ctypes.byref(a), int(tag), _ptr(out["Y2"]),
                                                _ptr(out["len"]), _stream(stream)))
        return out

    def pair_paths(self, s, t, omega, seed, root=-1, *, B=1, check=True, lanes=0, sample_begin=0, n_total=0,
                   mode=0, pool=0, group=0, stream_id=0, qid=0, timeout_s=0.0, stream=None):
        """Loop-included paths from node pairs (lap_pair_paths): V [B][n_pairs][4],
        r and r_se [n_pairs], lv [n_pairs][3]."""
        s = np.ascontiguousarray(s, np.int32)
        t = np.ascontiguousarray(t, np.int32)
        if s.shape != t.shape or s.ndim != 1:
            raise ValueError("s and t must be 1-D arrays of equal length")
        a = self._args(omega, seed, root, 0, B, sample_begin, n_total, mode, pool, stream_id, qid, timeout_s,
                       group=group)
        P = len(s)
        out = dict(V=np.zeros((B, P, 4), np.int64), r=np.zeros(P), r_se=np.zeros(P), lv=np.zeros((P, 3)))
        _check(load_library().lap_pair_paths(self._h, ctypes.byref(a), _ptr(s), _ptr(t), P, int(bool(check)),
                                             int(lanes), _ptr(out["V"]), _ptr(out["r"]), _ptr(out["r_se"]), _ptr(out["lv"]),
                                             _stream(stream)))
        return out

    def landmark_traces(self, roots, omega, seed, stream=None):
        """Tr((I-P_v)^{-1}) estimate (mean Wilson draws) and its SE for each root."""
        roots = np.ascontiguousarray(roots, np.int32)
        tr = np.zeros(len(roots))
        se = np.zeros(len(roots))
        _check(load_library().lap_landmark_traces(self._h, _ptr(roots), len(roots), int(omega), int(seed), _ptr(tr),
                                                  _ptr(se), _stream(stream)))
        return tr, se

    def lv_rows(self, sources, omega, seed, root=-1, *, B=1, check=True, lanes=0, sample_begin=0, n_total=0,
                mode=0, pool=0, group=0, stream_id=0, qid=0, timeout_s=0.0, stream=None):
        """Whole rows of L_v^{-1} from loop-included paths (lap_lv_rows):
        Y [B][n_sources][n] departures per node, rows [n_sources][n]."""
        src = np.ascontiguousarray(sources, np.int32)
        if src.ndim != 1:
            raise ValueError("sources must be a 1-D array")
        a = self._args(omega, seed, root, 0, B, sample_begin, n_total, mode, pool, stream_id, qid, timeout_s,
                       group=group)
        out = dict(Y=np.zeros((B, len(src), self.n), np.int64), rows=np.zeros((len(src), self.n)))
        _check(load_library().lap_lv_rows(self._h, ctypes.byref(a), _ptr(src), len(src), int(bool(check)), int(lanes),
                                          _ptr(out["Y"]), _ptr(out["rows"]), _stream(stream)))
        return out

    def spantree_sample_bound(self, kind, eps, p_fail, root=-1):
        """Hoeffding sample size of Thm. 3 (kind 1, closeness) or Thm. 4 (kind 2,
        Kemeny) and the BFS depth it uses (lap_spantree_sample_bound)."""
        w = ctypes.c_double()
        d = ctypes.c_int32()
        _check(load_library().lap_spantree_sample_bound(self._h, int(root), int(kind), float(eps), float(p_fail),
                                                        ctypes.byref(w), ctypes.byref(d)))
        return w.value, d.value

    def last_stats(self):
        vals = [ctypes.c_int64() for _ in range(8)]
        _check(load_library().lap_last_stats(self._h, *[ctypes.byref(v) for v in vals]))
        keys = ("wilson_steps", "absorbed_steps", "trees", "iterations", "pops", "rescans", "idle_lane_rounds",
                "parked_lane_rounds")
        return {k: v.value for k, v in zip(keys, vals)}


class Batch:
    """Many (graph, root, omega) jobs in one persistent launch (lap_batch_*).

    jobs: list of dicts with n, src, dst and optionally keep_lcc, root,
    omega (n_samples), seed, stream_id, qid."""

    def __init__(self, jobs, stream=None):
        lib = load_library()
        self._keep = []
        arr = (C.BatchJob * len(jobs))()
        for i, j in enumerate(jobs):
            s = np.ascontiguousarray(j["src"], np.int32)
            d = np.ascontiguousarray(j["dst"], np.int32)
            self._keep += [s, d]
            arr[i] = C.BatchJob(n=int(j["n"]), n_edges=len(s), src=_ptr(s), dst=_ptr(d),
                                flags=(C.LAP_KEEP_LCC if j.get("keep_lcc") else 0)
                                | (C.LAP_DEGREE_ORDER if j.get("degree_order") else 0), root=int(j.get("root", -1)),
                                n_samples=int(j["omega"]), seed=int(j.get("seed", 1)),
                                stream=int(j.get("stream_id", 0)), qid=int(j.get("qid", 0)))
        h = ctypes.c_void_p()
        _check(lib.lap_batch_create(arr, len(jobs), _stream(stream), ctypes.byref(h)))
        self._h = h
        self._keep = None
        self.n_jobs = len(jobs)
        self.info = []
        for i in range(len(jobs)):
            n = ctypes.c_int64()
            nnz = ctypes.c_int64()
            r = ctypes.c_int32()
            _check(lib.lap_batch_job_info(h, i, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(r)))
            self.info.append(dict(n=n.value, nnz=nnz.value, root=r.value, omega=int(jobs[i]["omega"])))

    def close(self):
        if getattr(self, "_h", None):
            load_library().lap_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def tuning(pool=0, chunk_nodes=0, use_graph=True, timeout_s=0.0):
        return C.BatchTuning(pool=int(pool), chunk_nodes=int(chunk_nodes), use_graph=1 if use_graph else 0,
                             timeout_s=float(timeout_s) if timeout_s else _default_timeout())

    def run(self, tuning=None, stream=None):
        t = tuning if tuning is not None else self.tuning()
        _check(load_library().lap_batch_run(self._h, ctypes.byref(t), _stream(stream)))

    def autotune(self, stream=None):
        t = C.BatchTuning()
        ms = ctypes.c_double()
        _check(load_library().lap_batch_autotune(self._h, ctypes.byref(t), ctypes.byref(ms), _stream(stream)))
        return t, ms.value

    def result(self, job):
        inf = self.info[job]
        n, om = inf["n"], inf["omega"]
        r = dict(Y1=np.zeros(n, np.int64), Y2=np.zeros(n, np.int64), y1=np.zeros(om, np.int64),
                 len_uniform=np.zeros(om, np.int64), len_pi=np.zeros(om, np.int64), diag=np.zeros(n),
                 closeness=np.zeros(n), trace=np.zeros(1), kemeny=np.zeros(1), kemeny_se=np.zeros(1))
        o = C.BatchOut(y1=_ptr(r["Y1"]), y2=_ptr(r["Y2"]), y1_per_sample=_ptr(r["y1"]),
                       y2len_uniform=_ptr(r["len_uniform"]), y2len_pi=_ptr(r["len_pi"]), diag=_ptr(r["diag"]),
                       closeness=_ptr(r["closeness"]), trace=_ptr(r["trace"]), kemeny=_ptr(r["kemeny"]),
                       kemeny_se=_ptr(r["kemeny_se"]))
        _check(load_library().lap_batch_result(self._h, int(job), ctypes.byref(o)))
        return r

    def stats(self):
        v = [ctypes.c_int64() for _ in range(3)]
        _check(load_library().lap_batch_stats(self._h, *[ctypes.byref(x) for x in v]))
        return dict(wilson_steps=v[0].value, absorbed_steps=v[1].value, trees=v[2].value)


class Server:
    """Request loop over a resident Graph (lap_server_*)."""

    CLOSENESS, RESISTANCE, KEMENY = C.LAP_Q_CLOSENESS, C.LAP_Q_RESISTANCE, C.LAP_Q_KEMENY

    def __init__(self, graph: "Graph", seed=1, root=-1, stream_id=0, global_samples=0, arena_bytes=0,
                 launches=0, waves=0, items_per_launch=0, wilson_chunk=0, timeout_s=0.0, wilson_group=0,
                 wilson_slots=0, stream=None):
        cfg = C.ServerConfig(seed=int(seed), root=int(root), stream=int(stream_id), global_samples=int(global_samples),
                             arena_bytes=int(arena_bytes), launches=int(launches), waves=int(waves),
                             items_per_launch=int(items_per_launch), wilson_chunk=int(wilson_chunk),
                             timeout_s=float(timeout_s) if timeout_s else _default_timeout(),
                             wilson_group=int(wilson_group), wilson_slots=int(wilson_slots))
        h = ctypes.c_void_p()
        _check(load_library().lap_server_create(graph._h, ctypes.byref(cfg), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.graph = graph            # the graph must outlive the server

    def close(self):
        if getattr(self, "_h", None):
            load_library().lap_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, qid, kind, budget, u=0, w=0):
        _check(load_library().lap_server_submit(self._h, ctypes.byref(
            C.Query(qid=int(qid), kind=int(kind), u=int(u), w=int(w), budget=int(budget)))))

    def step(self, wait=False):
        _check(load_library().lap_server_step(self._h, 1 if wait else 0))

    def cancel(self, qid):
        _check(load_library().lap_server_cancel(self._h, int(qid)))

    def poll(self, max_results=4096):
        buf = (C.QueryResult * max_results)()
        k = ctypes.c_int32()
        _check(load_library().lap_server_poll(self._h, buf, max_results, ctypes.byref(k)))
        return [dict(qid=r.qid, kind=r.kind, status=r.status, value=r.value, se=r.se, t_submit=r.t_submit,
                     t_start=r.t_start, t_done=r.t_done) for r in buf[: k.value]]

    def pending(self):
        v = [ctypes.c_int64() for _ in range(3)]
        _check(load_library().lap_server_pending(self._h, *[ctypes.byref(x) for x in v]))
        return dict(queued=v[0].value, active=v[1].value, inflight=v[2].value)

    def globals(self):
        a = ctypes.c_double()
        b = ctypes.c_double()
        _check(load_library().lap_server_globals(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def run_all(self, timeout_s=600.0):
        """Drive the loop until every submitted query has completed."""
        import time as _t
        out = []
        t0 = _t.time()
        while True:
            self.step(wait=True)
            out += self.poll()
            p = self.pending()
            if p["queued"] == 0 and p["active"] == 0 and p["inflight"] == 0:
                out += self.poll()
                return out
            if _t.time() - t0 > timeout_s:
                raise TimeoutError("server did not drain")


def bench_gather(bytes_, lanes, mode, in_flight=1, flavor=0, stream=None):
    """Random 8-byte accesses per second over a working set (mode 0 independent
    with in_flight loads per lane and round, 1 chase, 2 independent loads plus
    one 8-byte store per round, 3 plus one 64-byte line store per round, loads
    and stores counted, 4 random 4-byte reads from a 64 KiB LDS table); flavor
    0 plain loads, 1 non-temporal,
    2 / 3 relaxed atomic loads at device / system scope."""
    r = ctypes.c_double()
    _check(load_library().lap_bench_gather(int(bytes_), int(lanes), int(mode), int(in_flight), int(flavor),
                                           ctypes.byref(r), _stream(stream)))
    return r.value


def diag_Ldagger(g: Graph, omega, seed, root=-1, se=True, stream=None):
    d = np.zeros(g.n)
    s = np.zeros(g.n) if se else None
    _check(load_library().lap_diag_Ldagger(g._h, int(root), int(omega), int(seed), _ptr(d), _ptr(s),
                                           _stream(stream)))
    return d, s


def ecc(g: Graph, omega, seed, root=-1, stream=None):
    c = np.zeros(g.n)
    tr = np.zeros(1)
    _check(load_library().lap_ecc(g._h, int(root), int(omega), int(seed), _ptr(c), _ptr(tr), _stream(stream)))
    return c, float(tr[0])


def kemeny(g: Graph, omega, seed, root=-1, stream=None):
    k = np.zeros(1)
    s = np.zeros(1)
    _check(load_library().lap_kemeny(g._h, int(root), int(omega), int(seed), _ptr(k), _ptr(s), _stream(stream)))
    return float(k[0]), float(s[0])
