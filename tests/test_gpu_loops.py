"""Loop-included paths of the Wilson stacks on the GPU against the oracle:
departures per node and per path are bit-exact (the same stack entries are
replayed), in every sampler form, on the small ER workload at full size and
on the mid workload."""
import numpy as np
import pytest

from oracle import csr, native
from tests.gpu_common import ba_edges, both, er256_edges, log, small_cases

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,group", [(2, 0), (3, 8), (1, 0)])
def test_loop_included_small_graphs_bit_exact(mode, group):
    for name, n, s, d in small_cases():
        og, hg = both(n, s, d)
        for root in sorted({0, csr.landmark(og), og.n - 1}):
            for tag in (1, 2):
                log(f"loops {name} root {root} tag {tag} mode {mode}")
                got = hg.loop_included(150, 3, tag, root, B=4, mode=mode, group=group, pool=11)
                exp = native.loop_included(og, root, 150, 3, tag, B=4)
                assert np.array_equal(got["Y2"], exp["Y2"]) and np.array_equal(got["len"], exp["len"])


def test_loop_included_er256_and_mid_workloads_bit_exact():
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    for tag in (1, 2):
        log(f"loops er256 tag {tag}")
        got = hg.loop_included(1 << 14, 1, tag, root, B=64)
        exp = native.loop_included(og, root, 1 << 14, 1, tag, B=64)
        assert np.array_equal(got["Y2"], exp["Y2"]) and np.array_equal(got["len"], exp["len"])
    n, s, d = ba_edges(100_000, 5, 0)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    for tag in (1, 2):
        log(f"loops ba100k tag {tag}")
        got = hg.loop_included(512, 1, tag, root, B=8)
        exp = native.loop_included(og, root, 512, 1, tag, B=8)
        assert np.array_equal(got["Y2"], exp["Y2"]) and np.array_equal(got["len"], exp["len"])


def test_loop_included_resume_and_argument_errors():
    from paper_2311_10290_amd import LapError
    n, s, d = ba_edges(5000, 3, 1)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    full = hg.loop_included(40, 2, 1, root, B=4, pool=6)
    a = hg.loop_included(15, 2, 1, root, B=4, sample_begin=0, n_total=40)
    b = hg.loop_included(25, 2, 1, root, B=4, sample_begin=15, n_total=40, mode=3, group=2)
    assert np.array_equal(a["Y2"] + b["Y2"], full["Y2"])
    assert np.array_equal(np.concatenate([a["len"], b["len"]]), full["len"])
    with pytest.raises(LapError):
        hg.loop_included(10, 1, 3)
