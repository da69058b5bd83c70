"""Parity at the sampler's documented limits, through the C ABI: node degree
below 2^24 (the adjacency record's degree field), at most 2^21 - 1 draws at
one node in one sample (the state word's count field), and sample indices
below 2^56 with the key words at their largest values.

  - Double star: nodes 0 and 1 joined to each other and to every other node
    of 2^24, so both have degree 2^24 - 1 and each draw there maps a 64-bit
    word onto the full 24-bit range.
  - Star: centre 0 with 2^24 - 1 leaves, rooted at leaf 1.  By the stack
    argument of Sec. 3.4 the centre draws K times in a sample, K the position
    of its first stack entry naming the root (geometric with mean 2^24 - 1);
    the sample's total is 2K + d - 2.  At Philox seed 1, sample 2 passes the
    count limit and sample 52 comes within 6% of it."""
import numpy as np
import pytest

from oracle import csr, native
from tests.gpu_common import log

pytestmark = pytest.mark.gpu

D = (1 << 24) - 1
KMAX = (1 << 21) - 1


def _same(a, b, keys):
    for k in keys:
        assert a[k] is not None and b[k] is not None, k
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_max_degree_double_star_bit_exact():
    from paper_2311_10290_amd import Graph
    n = 1 << 24
    rest = np.arange(2, n, dtype=np.int32)
    src = np.concatenate([np.zeros(1 + len(rest), np.int32), np.ones(len(rest), np.int32)])
    dst = np.concatenate([np.ones(1, np.int32), rest, rest])
    log("double star 2^24: building both graphs")
    og = csr.build_csr(n, src, dst)
    hg = Graph(n, src, dst)
    assert og.deg[0] == D and og.deg[1] == D and hg.max_deg == D
    omega, seed, root = 4, 3, 1
    w = native.wilson(og, root, omega, seed, B=2, keep=[0, 3])
    a = native.absorbed(og, root, omega, seed, 1, B=2)
    exp = dict(Y1=w["Y1"], y1=w["y1"], next=w["next"], draws=w["draws"], Y2=a["Y2"], len_uniform=a["len"])
    assert exp["draws"][:, 0].max() >= 1
    for mode, group in ((2, 0), (3, 8)):
        log(f"double star 2^24: mode {mode} group {group}")
        got = hg.sample_forests(omega, seed, root, y2=True, B=2, keep=[0, 3], mode=mode, group=group)
        _same(got, exp, ["Y1", "y1", "next", "draws", "Y2", "len_uniform"])
    hg.close()


def test_star_draw_limit_reported_and_samples_below_it_exact():
    from paper_2311_10290_amd import Graph, LapError
    n = D + 1
    src = np.zeros(D, np.int32)
    dst = np.arange(1, n, dtype=np.int32)
    log("star 2^24 - 1 leaves: building both graphs")
    og = csr.build_csr(n, src, dst)
    hg = Graph(n, src, dst)
    root, seed, total = 1, 1, 64

    def oracle(i):
        w = native.wilson(og, root, total, seed, sample_begin=i, n_samples=1, B=1, keep=[i])
        return w, (int(w["y1"][0]) - D + 2) // 2

    log("star: oracle samples 2, 5, 52")
    _, k2 = oracle(2)
    w5, k5 = oracle(5)
    w52, k52 = oracle(52)
    assert k2 > KMAX and k5 < 10_000 and KMAX * 9 // 10 < k52 <= KMAX
    assert w52["draws"][0][0] == k52
    log("star: sample 2 (over the count limit), wave form")
    with pytest.raises(LapError) as ei:
        hg.sample_forests(1, seed, root, sample_begin=2, n_total=total, mode=2, timeout_s=300)
    assert ei.value.code == -5 and "draws at node 0" in str(ei.value)
    # the failed call leaves no trace in the next ones
    for i, w, mode, group in ((5, w5, 2, 0), (5, w5, 3, 8), (52, w52, 2, 0)):
        log(f"star: sample {i} mode {mode} group {group}")
        got = hg.sample_forests(1, seed, root, sample_begin=i, n_total=total, keep=[i], mode=mode, group=group,
                                timeout_s=300)
        _same(got, dict(Y1=w["Y1"], y1=w["y1"], next=w["next"], draws=w["draws"]), ["Y1", "y1", "next", "draws"])
    hg.close()


def test_extreme_keys_and_sample_indices_bit_exact():
    """The last 64 sample and walk indices below 2^56 (the counter field the
    keying leaves them) with the largest seed and stream id and a query id
    near 2^64: counts, kept trees and walk lengths equal the oracle's in
    every sampler form; a run of 2^56 samples is refused."""
    from paper_2311_10290_amd import LapError
    from tests.gpu_common import both, er256_edges
    n, s, d = er256_edges()
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    total = (1 << 56) - 1
    begin = total - 64
    seed, stream, qid = (1 << 64) - 1, (1 << 32) - 1, (1 << 64) - 2
    keep = [begin, total - 1]
    w = native.wilson(og, root, total, seed, stream=stream, qid=qid, sample_begin=begin, n_samples=64, B=4,
                      keep=keep)
    a1 = native.absorbed(og, root, 64, seed, 1, stream=stream, qid=qid, walk_begin=begin, omega_total=total, B=4)
    a2 = native.absorbed(og, root, 64, seed, 2, stream=stream, qid=qid, walk_begin=begin, omega_total=total,
                         want_y2=False)
    exp = dict(Y1=w["Y1"], y1=w["y1"], next=w["next"], draws=w["draws"], Y2=a1["Y2"], len_uniform=a1["len"],
               len_pi=a2["len"])
    assert exp["Y1"][:3].sum() == 0 and exp["Y1"][3].sum() > 0     # every sample falls in the last block
    for mode in (1, 2, 3, 4):
        log(f"extreme keys: mode {mode}")
        got = hg.sample_forests(64, seed, root, y2=True, y2_pi=True, B=4, keep=keep, sample_begin=begin,
                                n_total=total, mode=mode, stream_id=stream, qid=qid)
        _same(got, exp, ["Y1", "y1", "next", "draws", "Y2", "len_uniform", "len_pi"])
    with pytest.raises(LapError) as ei:
        hg.sample_forests(1, seed, root, n_total=1 << 56)
    assert ei.value.code == -1 and "2^56" in str(ei.value)
