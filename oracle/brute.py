"""Exhaustive ground states of small QUBOs (N <= 22).

Evaluates Eq. 13 on every T in {0,1}^N as the quadratic form
O(T) = a.T + 1/2 T^T b T (b symmetric, zero diagonal), in blocks of
assignments.  This is a different formulation from ``energy.qubo_energy``
(a pairwise loop), so each pins the other.
"""
from __future__ import annotations

import numpy as np


def ground_states(a: np.ndarray, b: np.ndarray, tol: float = 1e-12):
    """Return (E_min, list of minimising T vectors as int8 arrays)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = a.shape[0]
    if n > 22:
        raise ValueError("brute force limited to N <= 22")
    best = np.inf
    winners = []
    block = 1 << min(n, 16)
    bits = np.arange(n, dtype=np.int64)
    for start in range(0, 1 << n, block):
        idx = np.arange(start, min(start + block, 1 << n), dtype=np.int64)
        T = ((idx[:, None] >> bits[None, :]) & 1).astype(np.float64)
        e = T @ a + 0.5 * np.einsum("ki,ki->k", T @ b, T)
        m = e.min()
        if m < best - tol:
            winners = []
        best = min(best, m)
        if m <= best + tol:
            for k in np.nonzero(e <= best + tol)[0]:
                winners.append(T[k].astype(np.int8))
    return float(best), winners
