"""Pins for the oracle's random source: Philox4x64-10 against numpy's
implementation (a library routine), and the draw -> index mapping against
exact boundary arithmetic."""
import numpy as np
import pytest

from oracle import native

M64 = (1 << 64) - 1


def _numpy_block(ctr, key):
    # numpy's Philox increments its 256-bit counter before producing each block,
    # so the block for counter c is the first block of a generator set to c - 1.
    c = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & M64 for i in range(4)]
    bg = np.random.Philox(counter=np.array(words, np.uint64), key=np.array(key, np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [0, 0]),
    ([5, 7, 9, 11], [0x1234, 0x5678]),
    ([M64, M64, M64, M64], [M64, M64]),
    ([(2 << 56) | 4095, 831, 0, 17], [1, (3 << 32) | 245]),
    ([0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89],
     [0x452821E638D01377, 0xBE5466CF34E90C6C]),
])
def test_philox_matches_numpy(ctr, key):
    got = [int(x) for x in native.philox4x64_10(ctr, key)]
    assert got == _numpy_block(ctr, key)


def test_philox_random_counters_match_numpy():
    rng = np.random.default_rng(7)
    for _ in range(50):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.int64)]
        assert [int(x) for x in native.philox4x64_10(ctr, key)] == _numpy_block(ctr, key)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 7, 64, 1000, 162_743, 2**31 - 1])
def test_map_below_boundaries(d):
    # index j owns exactly the x with j*2^64 <= x*d < (j+1)*2^64
    for j in sorted({j for j in (0, 1, d // 2, d - 1) if j < d}):
        lo = -((-j << 64) // d)               # ceil(j * 2^64 / d)
        hi = (((j + 1) << 64) - 1) // d       # last x with x*d < (j+1)*2^64
        hi = min(hi, M64)
        assert native.map_below(lo, d) == j
        assert native.map_below(hi, d) == j
        if lo > 0:
            assert native.map_below(lo - 1, d) == j - 1


def test_map_below_small_exhaustive_shape():
    # with x = k * 2^60 (k = 0..15) and d = 3, indices follow floor(3k/16)
    for k in range(16):
        assert native.map_below(k << 60, 3) == (3 * k) // 16
