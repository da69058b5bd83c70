"""Helpers for the GPU parity tests (inputs from graphgen, expectations from the oracle)."""
import sys

import numpy as np

import graphgen as gg
from oracle import csr


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def er256_edges():
    s, d, _ = gg.erdos_renyi_connected(256, 0.05, 0)
    return 256, s, d


def ba_edges(n, m, seed=0):
    s, d = gg.barabasi_albert(n, m, seed)
    return n, s, d


def small_cases():
    out = []
    for name, args in [("diamond", ()), ("complete", (5,)), ("cycle", (7,)), ("path", (6,)), ("star", (6,)),
                       ("grid", (3, 4)), ("fig1_graph", ())]:
        s, d = getattr(gg, name)(*args)
        n = int(max(s.max(), d.max())) + 1
        out.append((name, n, s, d))
    return out


def both(n, s, d, keep_lcc=False, degree_order=False):
    """(oracle graph, HIP graph) built from the same edge list."""
    from paper_2311_10290_amd import Graph
    return (csr.build_csr(n, s, d, keep_lcc=keep_lcc, degree_order=degree_order),
            Graph(n, s, d, keep_lcc=keep_lcc, degree_order=degree_order))
