"""Pin of the oracle's Wilson sampler on stars by the stack argument of
Sec. 3.4, using only the generator and the index map (both pinned on their
own against numpy's Philox and exact boundary arithmetic).

Root a leaf r.  Every other leaf has the centre as its only neighbour, so
its stack names the centre at every level.  An entry of the centre's stack
that names a leaf l != r therefore closes the cycle centre -> l -> centre,
which is popped together with l's top entry.  The first entry naming r is
never popped.  Hence, per sample:
  - the centre draws K times, K the position of its first entry naming r;
  - a leaf l != r draws once, plus once per earlier centre entry naming l;
  - the tree is the star with the centre's arrow on r;
  - the sample's total is 2K + d - 2 for d leaves."""
import numpy as np
import pytest

from oracle import csr, native


def _centre_entry(sample, k, seed, root, d):
    # Wilson draws: counter (sample, node, level, query id 0), key (seed,
    # stream 0 << 32 | root); the centre is node 0, its neighbours 1..d
    x = native.philox4x64_10([sample, 0, k, 0], [seed, root])[0]
    return 1 + native.map_below(int(x), d)


def _star(d):
    n = d + 1
    return n, csr.build_csr(n, np.zeros(d, np.int32), np.arange(1, n, dtype=np.int32))


@pytest.mark.parametrize("d,r,seed", [(7, 3, 1), (200, 1, 5), (1000, 1000, 2)])
def test_star_counts_and_trees_follow_the_stack_argument(d, r, seed):
    n, og = _star(d)
    omega = 12
    got = native.wilson(og, r, omega, seed, keep=list(range(omega)), B=1)
    total = np.zeros(n, np.int64)
    for i in range(omega):
        draws = np.ones(n, np.int64)
        draws[r] = 0
        k = 0
        while (leaf := _centre_entry(i, k, seed, r, d)) != r:
            draws[leaf] += 1
            k += 1
        K = k + 1
        draws[0] = K
        nxt = np.zeros(n, np.int64)
        nxt[0], nxt[r] = r, -1
        assert np.array_equal(got["draws"][i], draws), i
        assert np.array_equal(got["next"][i], nxt), i
        assert got["y1"][i] == 2 * K + d - 2
        total += draws
    assert np.array_equal(got["Y1"][0], total)


def test_star_with_the_centre_as_root_draws_once_per_leaf():
    """Root the centre: every leaf's first entry names the tree."""
    d = 50
    n, og = _star(d)
    got = native.wilson(og, 0, 5, 3, keep=[0, 4], B=1)
    assert np.all(got["y1"] == d)
    assert np.array_equal(got["draws"], np.tile(np.r_[0, np.ones(d, np.int32)], (2, 1)))
    assert np.array_equal(got["next"], np.tile(np.r_[-1, np.zeros(d, np.int32)], (2, 1)))
