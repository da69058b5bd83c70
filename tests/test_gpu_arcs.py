"""The arc form of the Wilson samplers.  On graphs whose column array is at
least 64 MB the library also keeps, per column slot, the arc record {target,
target's adjacency record}; a draw then reads the record of its drawn slot
and an arrival loads only the target's state word.  The draws are the same
keyed draws, so every count and kept tree must equal the oracle's bit for bit
in the wave and workgroup forms (R-MAT scale 19, edge factor 32, largest
component: 29.7 M column entries, 113 MB)."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr
from tests.gpu_common import both, log
from tests.test_gpu_parity import _oracle_counts, _same

pytestmark = pytest.mark.gpu

WAVE, GROUP = 2, 3


@pytest.fixture(scope="module")
def rmat19():
    s, d = gg.rmat(19, 32, seed=5)
    og, hg = both(1 << 19, s, d, keep_lcc=True)
    assert og.nnz * 4 >= 64 << 20     # the library builds arc records for it
    return og, hg


@pytest.mark.parametrize("mode,group,pool", [(WAVE, 0, 0), (WAVE, 0, 7), (GROUP, 2, 0), (GROUP, 4, 5), (GROUP, 8, 0)])
def test_arc_form_bit_exact(rmat19, mode, group, pool):
    og, hg = rmat19
    root = csr.landmark(og)
    omega = 40
    keep = [0, 17, omega - 1]
    log(f"arcs rmat19 n={og.n} mode {mode} group {group} pool {pool}")
    got = hg.sample_forests(omega, 3, root, B=4, keep=keep, y2=True, y2_pi=True, mode=mode, group=group, pool=pool)
    exp = _oracle_counts(og, root, omega, 3, B=4, keep=keep)
    _same(got, exp, ["Y1", "y1", "next", "draws", "Y2", "len_uniform", "len_pi"])


@pytest.mark.parametrize("mode,group", [(WAVE, 0), (GROUP, 8)])
def test_arc_form_degree_ordered_graph(mode, group):
    """The same graph numbered by decreasing degree (the layout of the large
    workload): still bit-exact against the oracle on the same numbering."""
    s, d = gg.rmat(19, 32, seed=5)
    og, hg = both(1 << 19, s, d, keep_lcc=True, degree_order=True)
    root = csr.landmark(og)
    assert root == 0
    log(f"arcs rmat19 degree order mode {mode} group {group}")
    got = hg.sample_forests(40, 3, root, B=4, keep=[0, 39], y2=True, y2_pi=True, mode=mode, group=group)
    exp = _oracle_counts(og, root, 40, 3, B=4, keep=[0, 39])
    _same(got, exp, ["Y1", "y1", "next", "draws", "Y2", "len_uniform", "len_pi"])


def test_arc_form_other_root_and_rotated_scan(rmat19):
    og, hg = rmat19
    root = int(np.argsort(og.deg)[-7])      # a hub that is not the landmark
    exp = _oracle_counts(og, root, 24, 9, B=3, keep=[5], uniform=False, pi=False)
    for mode, group, sched in ((WAVE, 0, 12345), (GROUP, 8, og.n - 3)):
        log(f"arcs rmat19 root {root} mode {mode} schedule {sched}")
        got = hg.sample_forests(24, 9, root, B=3, keep=[5], mode=mode, group=group, schedule=sched)
        _same(got, exp, ["Y1", "y1", "next", "draws"])
