"""ctypes declarations mirroring include/lap.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblap.so")

LAP_OK, LAP_EINVAL, LAP_ENOTCONN, LAP_ENOMEM, LAP_EDEVICE, LAP_ERANGE, LAP_ECANCELED = 0, -1, -2, -3, -4, -5, -6
LAP_KEEP_LCC, LAP_DEGREE_ORDER = 1, 2
LAP_WANT_Y1, LAP_WANT_Y2_UNIFORM, LAP_WANT_Y2_PI, LAP_WANT_PER_SAMPLE, LAP_OUT_DEVICE = 1, 2, 4, 8, 16
LAP_MODE_AUTO, LAP_MODE_LANE, LAP_MODE_WAVE, LAP_MODE_GROUP, LAP_MODE_LDS = 0, 1, 2, 3, 4

# every symbol include/lap.h declares
EXPORTS = [
    "lap_build_csr", "lap_graph_info", "lap_graph_copy_csr", "lap_graph_free",
    "lap_sample_forests", "lap_sample_forests_noalloc", "lap_estimate", "lap_diag_Ldagger", "lap_ecc", "lap_kemeny",
    "lap_last_error", "lap_prof_enable", "lap_prof_reset", "lap_prof_read", "lap_last_stats",
    "lap_bench_gather",
    "lap_batch_create", "lap_batch_job_info", "lap_batch_run", "lap_batch_autotune", "lap_batch_result",
    "lap_batch_stats", "lap_batch_free", "lap_landmark_traces", "lap_spantree", "lap_spantree_estimate",
    "lap_loop_included", "lap_pair_paths", "lap_lv_rows", "lap_spantree_sample_bound",
    "lap_server_create", "lap_server_submit", "lap_server_step", "lap_server_cancel", "lap_server_poll",
    "lap_server_pending",
    "lap_server_globals", "lap_server_free",
]
LAP_Q_CLOSENESS, LAP_Q_RESISTANCE, LAP_Q_KEMENY = 0, 1, 2
LAP_SERVER_GLOBAL_QID = (1 << 64) - 1


class SampleArgs(ctypes.Structure):
    _fields_ = [
        ("n_samples", ctypes.c_int64), ("seed", ctypes.c_uint64), ("root", ctypes.c_int32),
        ("stream", ctypes.c_uint32), ("qid", ctypes.c_uint64), ("want", ctypes.c_uint32),
        ("n_blocks", ctypes.c_int32), ("sample_begin", ctypes.c_int64), ("n_total", ctypes.c_int64),
        ("mode", ctypes.c_int32), ("pool", ctypes.c_int32), ("timeout_s", ctypes.c_double),
        ("schedule", ctypes.c_int64), ("group", ctypes.c_int32), ("walks", ctypes.c_int32),
    ]


class Counts(ctypes.Structure):
    _fields_ = [
        ("y1", ctypes.c_void_p), ("y2", ctypes.c_void_p), ("y1_per_sample", ctypes.c_void_p),
        ("y2len_uniform", ctypes.c_void_p), ("y2len_pi", ctypes.c_void_p),
        ("keep_idx", ctypes.c_void_p), ("n_keep", ctypes.c_int64),
        ("next", ctypes.c_void_p), ("draws", ctypes.c_void_p),
    ]


class Estimates(ctypes.Structure):
    _fields_ = [
        ("diag", ctypes.c_void_p), ("diag_se", ctypes.c_void_p), ("lv_diag", ctypes.c_void_p),
        ("closeness", ctypes.c_void_p), ("trace", ctypes.c_void_p), ("kemeny", ctypes.c_void_p),
        ("kemeny_se", ctypes.c_void_p), ("kirchhoff", ctypes.c_void_p), ("rw_betweenness", ctypes.c_void_p),
    ]


class BatchJob(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("n_edges", ctypes.c_int64), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
        ("flags", ctypes.c_uint32), ("root", ctypes.c_int32), ("n_samples", ctypes.c_int64),
        ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint32), ("qid", ctypes.c_uint64),
    ]


class BatchTuning(ctypes.Structure):
    _fields_ = [("pool", ctypes.c_int32), ("chunk_nodes", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("timeout_s", ctypes.c_double)]


class BatchOut(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("y1", "y2", "y1_per_sample", "y2len_uniform", "y2len_pi", "diag",
                                                "closeness", "trace", "kemeny", "kemeny_se")]


class Query(ctypes.Structure):
    _fields_ = [("qid", ctypes.c_int64), ("kind", ctypes.c_int32), ("u", ctypes.c_int32), ("w", ctypes.c_int32),
                ("budget", ctypes.c_int64)]


class QueryResult(ctypes.Structure):
    _fields_ = [("qid", ctypes.c_int64), ("kind", ctypes.c_int32), ("status", ctypes.c_int32),
                ("value", ctypes.c_double), ("se", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("root", ctypes.c_int32), ("stream", ctypes.c_uint32),
                ("global_samples", ctypes.c_int64), ("arena_bytes", ctypes.c_int64), ("launches", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("items_per_launch", ctypes.c_int32), ("wilson_chunk", ctypes.c_int32),
                ("timeout_s", ctypes.c_double), ("wilson_group", ctypes.c_int32), ("wilson_slots", ctypes.c_int32)]


def declare(lib):
    P, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "lap_build_csr": ([i64, i64, P, P, u32, P, P], i32),
        "lap_graph_info": ([P, P, P, P, P], i32),
        "lap_graph_copy_csr": ([P, P, P, P], i32),
        "lap_graph_free": ([P], None),
        "lap_sample_forests": ([P, ctypes.POINTER(SampleArgs), ctypes.POINTER(Counts), P], i32),
        "lap_sample_forests_noalloc": ([P, ctypes.POINTER(SampleArgs), ctypes.POINTER(Counts), P], i32),
        "lap_estimate": ([P, ctypes.POINTER(SampleArgs), ctypes.POINTER(Estimates), P], i32),
        "lap_diag_Ldagger": ([P, i32, i64, u64, P, P, P], i32),
        "lap_ecc": ([P, i32, i64, u64, P, P, P], i32),
        "lap_kemeny": ([P, i32, i64, u64, P, P, P], i32),
        "lap_last_error": ([], ctypes.c_char_p),
        "lap_prof_enable": ([ctypes.c_int], i32),
        "lap_prof_reset": ([], i32),
        "lap_prof_read": ([ctypes.c_char_p, P, P], i32),
        "lap_last_stats": ([P, P, P, P, P, P, P, P, P], i32),
        "lap_bench_gather": ([i64, i64, i32, i32, i32, P, P], i32),
        "lap_batch_create": ([ctypes.POINTER(BatchJob), i32, P, P], i32),
        "lap_batch_job_info": ([P, i32, P, P, P], i32),
        "lap_batch_run": ([P, ctypes.POINTER(BatchTuning), P], i32),
        "lap_batch_autotune": ([P, ctypes.POINTER(BatchTuning), P, P], i32),
        "lap_batch_result": ([P, i32, ctypes.POINTER(BatchOut)], i32),
        "lap_batch_stats": ([P, P, P, P], i32),
        "lap_batch_free": ([P], None),
        "lap_landmark_traces": ([P, P, i32, i64, u64, P, P, P], i32),
        "lap_spantree": ([P, ctypes.POINTER(SampleArgs), P, P, P, P, P], i32),
        "lap_spantree_estimate": ([P, ctypes.POINTER(SampleArgs), P, P, P, P, P, P], i32),
        "lap_loop_included": ([P, ctypes.POINTER(SampleArgs), i32, P, P, P], i32),
        "lap_pair_paths": ([P, ctypes.POINTER(SampleArgs), P, P, i64, i32, i64, P, P, P, P, P], i32),
        "lap_lv_rows": ([P, ctypes.POINTER(SampleArgs), P, i64, i32, i64, P, P, P], i32),
        "lap_spantree_sample_bound": ([P, i32, i32, ctypes.c_double, ctypes.c_double, P, P], i32),
        "lap_server_create": ([P, ctypes.POINTER(ServerConfig), P, P], i32),
        "lap_server_submit": ([P, ctypes.POINTER(Query)], i32),
        "lap_server_step": ([P, i32], i32),
        "lap_server_cancel": ([P, i64], i32),
        "lap_server_poll": ([P, ctypes.POINTER(QueryResult), i32, P], i32),
        "lap_server_pending": ([P, P, P, P], i32),
        "lap_server_globals": ([P, P, P], i32),
        "lap_server_free": ([P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib
