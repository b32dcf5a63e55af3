"""The seeded operand generator (shared by oracle tests, GPU tests and the benchmark)."""
import numpy as np

import seeded_inputs as SI


def test_splitmix64_published_vectors():
    # first outputs for state 0, and for state 1234567, of the published splitmix64
    assert [int(x) for x in SI.splitmix64(0, 2)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]
    assert [int(x) for x in SI.splitmix64(1234567, 2)] == [6457827717110365317,
                                                           3203168211198807973]


def test_limbs_deterministic_and_split():
    a = SI.limbs(7, 9)
    assert a.dtype == np.uint32 and len(a) == 9
    assert np.array_equal(a, SI.limbs(7, 9))
    w = SI.splitmix64(7, 5)
    assert int(a[0]) == int(w[0]) & 0xFFFFFFFF and int(a[1]) == int(w[0]) >> 32


def test_batch_lengths_ranges():
    L = SI.batch_lengths(12345, 4096)
    assert len(L) == 4096
    for a, b in L:
        big, small = max(a, b), min(a, b)
        assert 1 <= small <= big <= (1 << 22) // 32 + 1
        assert big <= 8.0 * (small + 0.5)
