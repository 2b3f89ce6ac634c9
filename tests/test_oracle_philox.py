"""Pins of the oracle's Philox4x32-10 and of the SB initial state."""
import os

import numpy as np

from oracle.philox import initial_state, philox4x32_10, word_to_uniform

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        out = philox4x32_10(r[0], r[1], r[2], r[3], r[4], r[5])
        assert [int(v) for v in out] == r[6:10]


def test_philox_vectorised_matches_scalar():
    c0 = np.arange(5, dtype=np.uint64)
    out = philox4x32_10(c0, 7, 9, 11, 123, 456)
    for k in range(5):
        single = philox4x32_10(k, 7, 9, 11, 123, 456)
        assert all(int(out[w][k]) == int(single[w]) for w in range(4))


def test_uniform_map_endpoints_and_grid():
    # r >> 8 spans [0, 2^24): the map covers [-1/8, 1/8) on a 2^-26 grid
    assert word_to_uniform(0) == -0.125
    assert word_to_uniform(0xFFFFFFFF) == 0.125 - 2.0 ** -26
    assert word_to_uniform(1 << 31) == 0.0
    assert word_to_uniform(0xFF) == -0.125  # the low 8 bits are dropped


def test_initial_state_exact_in_fp32_and_layout():
    x, y = initial_state(37, 5, seed=0x1234_5678_9ABC_DEF0, event=3)
    assert x.shape == (37, 5) and y.shape == (37, 5)
    assert np.all(x.astype(np.float32).astype(np.float64) == x)
    assert np.all(np.abs(x) <= 0.125) and np.all(np.abs(y) <= 0.125)
    # counter = (spin, agent, event, 0), key = (seed lo, seed hi); x from word 0, y from word 1
    r = philox4x32_10(36, 4, 3, 0, 0x9ABC_DEF0, 0x1234_5678)
    assert x[36, 4] == word_to_uniform(int(r[0]))
    assert y[36, 4] == word_to_uniform(int(r[1]))
    # distinct agents and events draw distinct streams
    x2, _ = initial_state(37, 5, seed=0x1234_5678_9ABC_DEF0, event=4)
    assert not np.array_equal(x, x2)
    assert len(np.unique(x)) > 0.95 * x.size
