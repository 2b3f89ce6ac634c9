"""Philox4x32-10 counter-based generator and the SB initial state.

The paper does not say how the SB positions and momenta start (section
"Simulated Bifurcation" only fixes the equations of motion).  Both the
oracle and the HIP library therefore draw the start from one published
counter-based generator, Philox4x32 with 10 rounds (J. K. Salmon,
M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11), each side implementing it independently from that
definition.

Round: with multipliers M0, M1 and the current key (k0, k1),
    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2      (32x32 -> 64-bit)
    c' = (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)
and the key is bumped by the Weyl constants (W0, W1) between rounds.

Initial state (a reading; see the module docstring of ``sb``): for spin i,
agent m, event e and 64-bit seed s, counter = (i, m, e, 0) and
key = (s mod 2^32, s >> 32).  Output words r0, r1 give
    x0 = ((r0 >> 8) - 2^23) * 2^-26,   y0 = ((r1 >> 8) - 2^23) * 2^-26,
uniform on [-1/8, 1/8) on a 2^-26 grid: exactly representable in FP32 and
FP64, so the FP32 device path and this FP64 oracle start bit-identically.
"""
from __future__ import annotations

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x32-10.  Counter words are arrays (broadcast
    together); key words are Python ints.  Returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & _MASK32
    k1 = int(k1) & _MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    sh = np.uint64(32)
    lo_mask = np.uint64(_MASK32)
    for rnd in range(10):
        p0 = m0 * c0            # < 2^64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> sh, p0 & lo_mask
        hi1, lo1 = p1 >> sh, p1 & lo_mask
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        if rnd < 9:
            k0 = (k0 + PHILOX_W0) & _MASK32
            k1 = (k1 + PHILOX_W1) & _MASK32
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def word_to_uniform(r) -> np.ndarray:
    """((r >> 8) - 2^23) * 2^-26 as FP64 (exact)."""
    r = np.asarray(r, dtype=np.int64)
    return ((r >> 8) - (1 << 23)).astype(np.float64) * 2.0 ** -26


def initial_state(n: int, agents: int, seed: int, event: int = 0, spins=None):
    """x0, y0 of shape [n, agents] (spin-major, agents contiguous), FP64.
    With `spins` (an index array) only those spins' rows are drawn."""
    i = (np.arange(n, dtype=np.uint64) if spins is None
         else np.asarray(spins, dtype=np.uint64))[:, None]
    m = np.arange(agents, dtype=np.uint64)[None, :]
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    r0, r1, _, _ = philox4x32_10(i, m, np.uint64(event), np.uint64(0),
                                 seed & _MASK32, seed >> 32)
    return word_to_uniform(r0), word_to_uniform(r1)
