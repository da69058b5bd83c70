"""Shared helpers for the oracle tests: small graphs and golden-file readers."""
import os

import numpy as np

import graphgen as gg
from oracle import csr

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def graph(name, *args, keep_lcc=False):
    src, dst = getattr(gg, name)(*args)
    n = int(max(src.max(), dst.max())) + 1
    return csr.build_csr(n, src, dst, keep_lcc=keep_lcc)


def er256():
    src, dst, _ = gg.erdos_renyi_connected(256, 0.05, 0)
    return csr.build_csr(256, src, dst)


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, rest = line.split(None, 1)
            rows.append((tag, rest))
    return rows


def ints(s):
    return [int(x) for x in s.split()]
