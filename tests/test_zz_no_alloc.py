"""lap_sample_forests_noalloc (the entry point whose scratch is a fixed device
array) against lap_sample_forests: the same counts bit for bit, on two calls
in a row where the second has a smaller graph and sample count (the scratch
keeps the first call's contents), in the wave, lane, workgroup and LDS forms;
sizes beyond the fixed scratch are refused before anything runs."""
import numpy as np
import pytest

import graphgen as gg
from tests.gpu_common import log

pytestmark = pytest.mark.gpu

KEYS = ["Y1", "Y2", "y1", "len_uniform", "len_pi", "next", "draws"]


def _compare(hg, omega, seed, root, B, keep, mode=0, group=0):
    ref = hg.sample_forests(omega, seed, root, y2=True, y2_pi=True, B=B, keep=keep, mode=mode, group=group)
    got = hg.sample_forests_noalloc(omega, seed, root, y2=True, y2_pi=True, B=B, keep=keep, mode=mode,
                                    group=group)
    for k in KEYS:
        assert np.array_equal(got[k].cpu().numpy(), ref[k]), k


def test_noalloc_equals_plain_call_twice_second_smaller():
    import torch
    from paper_2311_10290_amd import Graph
    torch.cuda.set_device(0)
    n, s, d = 30_000, *gg.barabasi_albert(30_000, 4, 3)
    big = Graph(n, s, d)
    log("noalloc: BA 30000, 700 samples (wave form)")
    _compare(big, 700, 3, -1, B=8, keep=[0, 350, 699])
    s, d, _ = gg.erdos_renyi_connected(256, 0.05, 0)
    small = Graph(256, s, d)
    log("noalloc: ER 256, 300 samples after the larger call")
    _compare(small, 300, 1, -1, B=4, keep=[0, 299])
    log("noalloc: ER 256, lane, LDS and workgroup forms")
    _compare(small, 200, 2, 7, B=3, keep=[5], mode=1)
    _compare(small, 300, 1, -1, B=4, keep=[0, 299], mode=4)
    _compare(small, 90, 4, -1, B=2, keep=[89], mode=3, group=4)
    log("noalloc: BA 30000 again, fewer samples")
    _compare(big, 129, 8, -1, B=1, keep=[128])


def test_noalloc_refuses_sizes_beyond_its_scratch():
    import torch
    from paper_2311_10290_amd import Graph, LapError
    torch.cuda.set_device(0)
    s, d, _ = gg.erdos_renyi_connected(256, 0.05, 0)
    g = Graph(256, s, d)
    with pytest.raises(LapError) as ei:
        g.sample_forests_noalloc(5000, 1, B=4097)
    assert ei.value.code == -5
    # a star of 9 million nodes: one slot of walk state would need 72 MB
    m = 9_000_000
    star = Graph(m, np.zeros(m - 1, np.int32), np.arange(1, m, dtype=np.int32))
    log("noalloc: star of 9M nodes is refused")
    with pytest.raises(LapError) as ei:
        star.sample_forests_noalloc(4, 1)
    assert ei.value.code == -5
    # walks alone need no walk state and still run on the large graph
    got = star.sample_forests_noalloc(64, 1, y1=False, per_sample=False, y2_pi=True)
    ref = star.sample_forests(64, 1, y1=False, per_sample=False, y2_pi=True)
    assert np.array_equal(got["len_pi"].cpu().numpy(), ref["len_pi"])
    # and the small graph still works after the refusals
    _compare(g, 64, 5, -1, B=2, keep=[63])
