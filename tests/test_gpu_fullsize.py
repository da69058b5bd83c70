"""Parity at the full size of the mid workload (Barabasi-Albert n = 100,000,
m = 5, root = max degree, 2^12 samples) in the launch configuration the
benchmark uses: every integer count over all samples is compared with the
oracle (which runs the same samples on the host cores), plus per-node
next/draws of sampled trees."""
import numpy as np
import pytest

from oracle import csr, native
from tests.gpu_common import ba_edges, both, log

pytestmark = pytest.mark.gpu


def test_ba100k_counts_bit_exact():
    n, s, d = ba_edges(100_000, 5, 0)
    og, hg = both(n, s, d)
    root = csr.landmark(og)
    omega = 1 << 12
    keep = [0, 1, 2048, omega - 1]
    log("ba100k: HIP path")
    got = hg.sample_forests(omega, 1, root, y2=True, y2_pi=True, B=64, keep=keep)
    log("ba100k: oracle Wilson")
    w = native.wilson(og, root, omega, 1, B=64, keep=keep)
    assert np.array_equal(got["y1"], w["y1"])
    assert np.array_equal(got["Y1"], w["Y1"])
    assert np.array_equal(got["next"], w["next"]) and np.array_equal(got["draws"], w["draws"])
    log("ba100k: oracle absorbed walks")
    a = native.absorbed(og, root, omega, 1, 1, B=64)
    assert np.array_equal(got["Y2"], a["Y2"]) and np.array_equal(got["len_uniform"], a["len"])
    p = native.absorbed(og, root, omega, 1, 2, want_y2=False)
    assert np.array_equal(got["len_pi"], p["len"])


def test_rmat22_large_workload_counts_bit_exact():
    """The large workload at full size: R-MAT scale 22 (edge factor 16,
    a/b/c/d = .57/.19/.19/.05) largest component, root = max degree, 512
    samples, in the benchmark's launch configuration (automatic form: the
    workgroup sampler).  Every sample's total draws, the per-block counts and
    two sampled trees equal the oracle's."""
    import graphgen as gg
    from tests.gpu_common import both as _both
    s, d = gg.rmat(22, 16, seed=0)
    log("rmat22: CSR (both sides)")
    og, hg = _both(1 << 22, s, d, keep_lcc=True)
    del s, d
    root = csr.landmark(og)
    omega = 512
    keep = [0, omega - 1]
    log(f"rmat22 n={og.n}: HIP path")
    got = hg.sample_forests(omega, 1, root, B=64, keep=keep)
    log("rmat22: oracle Wilson")
    w = native.wilson(og, root, omega, 1, B=64, keep=keep)
    assert np.array_equal(got["y1"], w["y1"])
    assert np.array_equal(got["Y1"], w["Y1"])
    assert np.array_equal(got["next"], w["next"]) and np.array_equal(got["draws"], w["draws"])
