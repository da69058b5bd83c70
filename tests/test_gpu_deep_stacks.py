"""Nodes that draw more than 255 times in one sample.

The wave and workgroup samplers keep a walker's path in LDS with one byte per
entry for the node's draw count; a node that draws for the 256th time moves
the walker to memory mode (the path written out as next/draw words, every
later draw stored and next pointers followed).  Expected draws at u are
N_uu = d_u r(u, v) (Sec. 3.3), so the path P_200 rooted at one end (N_uu = 2u
inside the path) and the 2 x 100 ladder rooted at a corner reach that branch
in most samples.  Every count, both walk kinds and every kept tree must equal
the oracle's bit for bit in the lane, wave, workgroup and LDS forms, and the
oracle's own draws show that the branch was taken (the LDS form keeps 21-bit
draw counts in its state words and has no such branch; it runs the same
cases)."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr
from tests.gpu_common import log
from tests.test_gpu_parity import _oracle_counts, _same

pytestmark = pytest.mark.gpu

LANE, WAVE, GROUP, LDS = 1, 2, 3, 4
OMEGA = 64


def _graph(name, *args):
    s, d = getattr(gg, name)(*args)
    n = int(max(s.max(), d.max())) + 1
    return n, s, d


CASES = [("path200", _graph("path", 200)), ("ladder2x100", _graph("grid", 2, 100))]
FORMS = [(LANE, 0), (WAVE, 0), (GROUP, 2), (GROUP, 4), (GROUP, 8), (LDS, 0)]


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_more_than_255_draws_at_a_node_bit_exact(case):
    from paper_2311_10290_amd import Graph
    name, (n, s, d) = CASES[case]
    og = csr.build_csr(n, s, d)
    hg = Graph(n, s, d)
    root = 0
    keep = list(range(OMEGA))
    exp = _oracle_counts(og, root, OMEGA, 5, B=4, keep=keep)
    deep = int((exp["draws"].max(axis=1) > 255).sum())
    log(f"{name}: {deep} of {OMEGA} samples draw more than 255 times at some node "
        f"(max {int(exp['draws'].max())})")
    assert deep >= 8
    for mode, group in FORMS:
        log(f"{name} mode {mode} group {group}")
        got = hg.sample_forests(OMEGA, 5, root, B=4, keep=keep, y2=True, y2_pi=True, mode=mode, group=group,
                                pool=16)
        _same(got, exp, ["Y1", "y1", "next", "draws", "Y2", "len_uniform", "len_pi"])
