"""Pins for the oracle's FP64 estimator assembly: exact expectations plugged
into the assembly give the dense ground truth (the assembly is the
algebra of Alg. 2 / Alg. 4), and sampled estimates at the small ER workload
are within the statistical tolerance of the dense values."""
import math

import numpy as np
import pytest

from oracle import csr, dense, estimators, native
from tests.oracle_fixtures import er256, graph


@pytest.mark.parametrize("make", [lambda: graph("diamond"), lambda: graph("grid", 3, 4), er256])
def test_assembly_of_exact_expectations_is_exact(make):
    g = make()
    L = dense.laplacian(g)
    Ld = dense.pinv_eigh(L)
    for v in (0, csr.landmark(g)):
        e = dense.expected_counts(g, v)
        omega = 1
        # plug real-valued expectations in place of the integer counts
        diag = estimators.diag_ldagger(e["draws"], e["visits_uniform"], omega, g.deg)
        assert np.allclose(diag, np.diag(Ld), atol=1e-10)
        c, tr = estimators.closeness(diag)
        assert np.allclose(c, dense.closeness(Ld), rtol=1e-10)
        assert e["total"] - e["len_stationary"] == pytest.approx(dense.kemeny_spectral(g), rel=1e-10)


def test_block_sizes():
    assert estimators.block_sizes(100, 7).tolist() == [15, 14, 14, 15, 14, 14, 14]
    assert estimators.block_sizes(64, 64).tolist() == [1] * 64


def test_kemeny_estimator_and_se():
    est, se = estimators.kemeny([10, 12, 14], [1, 2, 3])
    assert est == pytest.approx(10.0)
    assert se == pytest.approx(np.std([9, 10, 11], ddof=1) / math.sqrt(3))


def _er256_run(seed, omega=1 << 14, B=64):
    g = er256()
    v = csr.landmark(g)
    w = native.wilson(g, v, omega, seed, B=B)
    a1 = native.absorbed(g, v, omega, seed, 1, B=B)
    a2 = native.absorbed(g, v, omega, seed, 2, want_y2=False)
    diag, se = estimators.diag_ldagger_blocks(w["Y1"], a1["Y2"], omega, g.deg)
    k, kse = estimators.kemeny(w["y1"], a2["len"])
    return g, diag, se, k, kse


def test_er256_estimates_within_standard_errors():
    """Small ER workload: G(256, 0.05), root = max degree, 2^14 samples, Philox seed 1."""
    g, diag, se, k, kse = _er256_run(1)
    Ld = dense.pinv_eigh(dense.laplacian(g))
    z = (diag - np.diag(Ld)) / se
    # multiple-comparison rule: max |z| within the two-sided 0.27%/n Bonferroni
    # quantile (~4.55 at n = 256), and the bulk of the nodes within 3 SE
    assert np.abs(z).max() < 4.6
    assert (np.abs(z) < 3).mean() >= 0.97
    assert abs(k - dense.kemeny_spectral(g)) < 3 * kse


def test_er256_relative_error_target_over_seeds():
    """The 1e-2 relative target for Kemeny's constant and the mean closeness
    error holds for the typical run: the median over five seeds is below it.
    (Seed 1 alone is a ~2-sigma run: kappa 1.1%, mean closeness 1.2%.)"""
    g = er256()
    Ld = dense.pinv_eigh(dense.laplacian(g))
    c_true = dense.closeness(Ld)
    k_true = dense.kemeny_spectral(g)
    cs, ks = [], []
    for seed in range(1, 6):
        _, diag, _, k, _ = _er256_run(seed)
        c, _ = estimators.closeness(diag)
        cs.append(float(np.mean(np.abs(c - c_true) / c_true)))
        ks.append(abs(k - k_true) / k_true)
    assert np.median(cs) < 1e-2
    assert np.median(ks) < 1e-2


def _er256_loop_run(seed, omega=1 << 14, B=64):
    """The same Wilson samples, with the absorbed-walk counts taken from
    their loop-included paths (Sec. 3.4) instead of fresh walks."""
    g = er256()
    v = csr.landmark(g)
    w = native.wilson(g, v, omega, seed, B=B)
    l1 = native.loop_included(g, v, omega, seed, 1, B=B)
    l2 = native.loop_included(g, v, omega, seed, 2)
    diag, se = estimators.diag_ldagger_blocks(w["Y1"], l1["Y2"], omega, g.deg)
    k, kse = estimators.kemeny(w["y1"], l2["len"])
    return g, diag, se, k, kse


def test_er256_loop_included_estimates_within_standard_errors():
    g, diag, se, k, kse = _er256_loop_run(1)
    Ld = dense.pinv_eigh(dense.laplacian(g))
    z = (diag - np.diag(Ld)) / se
    assert np.abs(z).max() < 4.6
    assert (np.abs(z) < 3).mean() >= 0.97
    assert abs(k - dense.kemeny_spectral(g)) < 3 * kse


def test_er256_relative_error_target_at_seed_1():
    """The 1e-2 relative target on the small ER workload at the configured
    Philox seed 1.  The fresh-walk estimator misses it there (a ~2-sigma run:
    kappa 1.1%, mean closeness 1.2%); the loop-included estimator on the same
    2^14 Wilson samples meets it for kappa, the mean and the maximum closeness
    error, because its walk counts share the samples' stacks and its errors
    largely cancel."""
    g = er256()
    Ld = dense.pinv_eigh(dense.laplacian(g))
    c_true = dense.closeness(Ld)
    k_true = dense.kemeny_spectral(g)
    _, diag, _, k, _ = _er256_run(1)
    c, _ = estimators.closeness(diag)
    assert abs(k - k_true) / k_true > 1e-2                       # the fresh-walk miss, as measured
    assert np.mean(np.abs(c - c_true) / c_true) > 1e-2
    _, diag, _, k, kse = _er256_loop_run(1)
    c, _ = estimators.closeness(diag)
    rel = np.abs(c - c_true) / c_true
    assert abs(k - k_true) / k_true < 1e-2
    assert rel.mean() < 1e-2 and rel.max() < 1e-2
