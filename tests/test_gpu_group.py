"""The workgroup form of the Wilson sampler (2, 4 or 8 wavefronts -- 128 to
512 walkers -- per sample) against the oracle: bit-exact counts and kept
trees on tiny graphs (far fewer nodes than walkers), the small ER workload at
full size, ragged pools, rotated start scans, and the kernel's own time limit."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr
from tests.gpu_common import ba_edges, both, er256_edges, log, small_cases
from tests.test_gpu_parity import _oracle_counts, _same

pytestmark = pytest.mark.gpu

GROUP = 3       # LAP_MODE_GROUP


@pytest.mark.parametrize("waves", [2, 4, 8])
def test_group_small_graphs_bit_exact(waves):
    for name, n, s, d in small_cases():
        og, hg = both(n, s, d)
        for root in sorted({0, csr.landmark(og), og.n - 1}):
            log(f"group {waves} small {name} root {root}")
            keep = [0, 1, 77, 299]
            got = hg.sample_forests(300, 9, root, B=4, keep=keep, mode=GROUP, group=waves, pool=7)
            exp = _oracle_counts(og, root, 300, 9, B=4, keep=keep, uniform=False, pi=False)
            _same(got, exp, ["Y1", "y1", "next", "draws"])


@pytest.mark.parametrize("waves", [2, 4, 8])
def test_group_er256_workload_bit_exact(waves):
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega = 1 << 14
    keep = [0, 5, 9999, omega - 1]
    log(f"group {waves} er256")
    got = hg.sample_forests(omega, 1, root, B=64, keep=keep, mode=GROUP, group=waves)
    exp = _oracle_counts(og, root, omega, 1, B=64, keep=keep, uniform=False, pi=False)
    _same(got, exp, ["Y1", "y1", "next", "draws"])


@pytest.mark.parametrize("pool", [1, 5, 300])
def test_group_pools_ragged_and_rotated_scans(pool):
    n, s, d = ba_edges(20_000, 3, 11)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega = 61
    exp = _oracle_counts(og, root, omega, 6, B=3, keep=[0, 60], uniform=False, pi=False)
    for waves, sched in ((8, 0), (4, 12345), (8, n - 1)):
        log(f"group {waves} pool {pool} schedule {sched}")
        got = hg.sample_forests(omega, 6, root, B=3, keep=[0, 60], mode=GROUP, group=waves, pool=pool,
                                schedule=sched)
        _same(got, exp, ["Y1", "y1", "next", "draws"])


def test_group_power_law_graph_with_a_long_tail():
    """R-MAT scale 15 (largest component): hubs, many degree-1 nodes, long
    walks -- the shape of the large workload at a size the oracle runs fast."""
    s, d = gg.rmat(15, 16, seed=2)
    og, hg = both(1 << 15, s, d, keep_lcc=True)
    root = csr.landmark(og)
    log(f"group rmat15 n={og.n}")
    got = hg.sample_forests(96, 2, root, B=2, keep=[3, 95], y2=True, mode=GROUP, group=8)
    exp = _oracle_counts(og, root, 96, 2, B=2, keep=[3, 95], pi=False)
    _same(got, exp, ["Y1", "y1", "next", "draws", "Y2", "len_uniform"])


def test_group_time_limit_is_reported_and_recovered():
    from paper_2311_10290_amd import LapError
    n, s, d = ba_edges(200_000, 3, 2)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    with pytest.raises(LapError) as ei:
        hg.sample_forests(64, 1, root, mode=GROUP, group=8, timeout_s=1e-4)
    assert ei.value.code == -5
    got = hg.sample_forests(8, 1, root, B=1, mode=GROUP, group=4)
    exp = _oracle_counts(og, root, 8, 1, B=1, uniform=False, pi=False)
    _same(got, exp, ["Y1", "y1"])


def test_group_argument_errors():
    from paper_2311_10290_amd import LapError
    n, s, d = er256_edges()
    _, hg = both(n, s, d)
    for g in (1, 3, 16, -2):
        with pytest.raises(LapError):
            hg.sample_forests(10, 1, mode=GROUP, group=g)
