"""The LDS lane form (LAP_MODE_LDS): one lane per sample with the CSR and the
samples' state words in LDS, for graphs of at most 1024 nodes.

Counts, both walk kinds and kept trees must equal the oracle's bit for bit on
graphs that take 64, 32 and 16 lanes per workgroup, with ragged sample counts,
with a pool small enough that each lane runs several samples one after
another, and when a run resumes in two halves.  Calls that read the trees
back from device memory refuse the form, graphs it cannot hold are refused
before anything runs, and its time limit stops the kernel normally."""
import numpy as np
import pytest

import graphgen as gg
from oracle import csr
from tests.gpu_common import both, log
from tests.test_gpu_parity import _oracle_counts, _same

pytestmark = pytest.mark.gpu

LDS = 4
ALL = ["Y1", "y1", "next", "draws", "Y2", "len_uniform", "len_pi"]


def _edges(name, *args):
    out = getattr(gg, name)(*args)
    s, d = out[0], out[1]
    n = int(max(s.max(), d.max())) + 1
    return n, s, d


def _lds_per_block():
    import torch
    props = torch.cuda.get_device_properties(0)
    return int(getattr(props, "shared_memory_per_block", 0) or 160 * 1024)


def _lanes(n, nnz, lds=None):
    """Samples per workgroup the library picks for a graph (64, 32 or 16)."""
    lds = lds or _lds_per_block()
    for lanes in (64, 32, 16):
        if 4 * ((n + 1) + (nnz + 1) // 2 + n * lanes) <= lds:
            return lanes
    return 0


# (name, graph, omega, pool): graphs of 64, 32 and 16 lanes per workgroup
CASES = [
    ("er256", _edges("erdos_renyi_connected", 256, 0.05, 0), 1000, 0),
    ("ba600", _edges("barabasi_albert", 600, 3, 2), 257, 0),
    ("path1000", _edges("path", 1000), 65, 0),
    ("er1000_dense", _edges("erdos_renyi_connected", 1000, 0.04, 3), 130, 0),
    ("grid32x32", _edges("grid", 32, 32), 200, 48),
    ("er256_pool", _edges("erdos_renyi_connected", 256, 0.05, 0), 700, 100),
]


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_lds_form_bit_exact(case):
    name, (n, s, d), omega, pool = CASES[case]
    og, hg = both(n, s, d)
    lanes = _lanes(og.n, og.nnz)
    assert lanes > 0
    for root in sorted({csr.landmark(og), og.n - 1}):
        keep = sorted({0, omega // 2, omega - 1})
        log(f"lds {name} n={og.n} nnz={og.nnz} lanes={lanes} root={root} omega={omega} pool={pool}")
        got = hg.sample_forests(omega, 7, root, y2=True, y2_pi=True, B=5, keep=keep, mode=LDS, pool=pool)
        exp = _oracle_counts(og, root, omega, 7, B=5, keep=keep)
        _same(got, exp, ALL)


def test_lds_form_lane_sizes_cover_all_three():
    log(f"LDS per workgroup: {_lds_per_block()} bytes")
    sizes = {_lanes(*(lambda og: (og.n, og.nnz))(csr.build_csr(*c[1])), lds=160 * 1024) for c in CASES}
    assert sizes == {64, 32, 16}


def test_lds_form_resumes_in_two_halves():
    n, s, d = _edges("erdos_renyi_connected", 256, 0.05, 0)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    log("lds resume er256")
    full = hg.sample_forests(1000, 2, root, y2=True, B=8, mode=LDS)
    a = hg.sample_forests(400, 2, root, y2=True, B=8, sample_begin=0, n_total=1000, mode=LDS)
    b = hg.sample_forests(600, 2, root, y2=True, B=8, sample_begin=400, n_total=1000, mode=2)
    assert np.array_equal(full["Y1"], a["Y1"] + b["Y1"])
    assert np.array_equal(full["y1"], np.concatenate([a["y1"], b["y1"]]))


def test_lds_form_degenerate_graphs():
    from paper_2311_10290_amd import Graph
    # one node: no walk, no draw
    g1 = Graph(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    got = g1.sample_forests(70, 1, 0, B=2, keep=[0, 69], mode=LDS)
    assert got["Y1"].sum() == 0 and got["y1"].sum() == 0
    assert got["next"][0, 0] == -1 and got["draws"][1, 0] == 0
    # two nodes and stars rooted at a leaf and at the centre
    for name, n, s, d in [("pair", 2, np.array([0], np.int32), np.array([1], np.int32)),
                          ("star9", *_edges("star", 9))]:
        og, hg = both(n, s, d)
        for root in range(og.n):
            log(f"lds degenerate {name} root {root}")
            got = hg.sample_forests(67, 3, root, y2=True, y2_pi=True, B=3, keep=[0, 66], mode=LDS)
            exp = _oracle_counts(og, root, 67, 3, B=3, keep=[0, 66])
            _same(got, exp, ALL)


def test_lds_form_estimate_matches_wave_form():
    n, s, d = _edges("erdos_renyi_connected", 256, 0.05, 0)
    _, hg = both(n, s, d)
    a = hg.estimate(2048, 5, -1, B=16, lv=True, derived=True, mode=LDS)
    b = hg.estimate(2048, 5, -1, B=16, lv=True, derived=True, mode=2)
    for k in ("diag", "diag_se", "lv_diag", "closeness", "trace", "kemeny", "kemeny_se", "kirchhoff",
              "rw_betweenness"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-15, err_msg=k)


def test_lds_form_refusals():
    from paper_2311_10290_amd import Graph, LapError
    # more than 1024 nodes, and 400 nodes whose 159,600 columns alone exceed LDS
    for name, args in (("barabasi_albert", (2000, 3, 1)), ("complete", (400,))):
        n, s, d = _edges(name, *args)
        big = Graph(n, s, d)
        with pytest.raises(LapError) as ei:
            big.sample_forests(64, 1, mode=LDS)
        assert ei.value.code == -5
        # the other forms still run there
        assert big.sample_forests(8, 1)["y1"].min() > 0
    n, s, d = _edges("erdos_renyi_connected", 256, 0.05, 0)
    g = Graph(n, s, d)
    for call in (lambda: g.spantree(64, 1, mode=LDS), lambda: g.loop_included(64, 1, 1, mode=LDS),
                 lambda: g.estimate(64, 1, mode=LDS, walks=1)):
        with pytest.raises(LapError) as ei:
            call()
        assert ei.value.code == -1
    # and those calls run in automatic mode
    g.loop_included(64, 1, 1)


def test_lds_form_time_limit_stops_normally():
    from paper_2311_10290_amd import LapError
    n, s, d = _edges("path", 1000)
    og, hg = both(n, s, d)
    log("lds time limit path1000")
    with pytest.raises(LapError) as ei:
        hg.sample_forests(4096, 1, 0, mode=LDS, timeout_s=1e-4)
    assert ei.value.code == -5 and "time limit" in str(ei.value)
    got = hg.sample_forests(64, 1, 0, B=2, mode=LDS)
    exp = _oracle_counts(og, 0, 64, 1, B=2, uniform=False, pi=False)
    _same(got, exp, ["Y1", "y1"])
