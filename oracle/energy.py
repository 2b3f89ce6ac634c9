"""FP64 QUBO objective (Eq. 13) and best-shot selection (Results section).

O(a, b, T) = sum_i a_i T_i + sum_i sum_{j<i} b_ij T_i T_j, evaluated in
FP64 with Neumaier-compensated summation.  The pair sum is taken as
sum over rows i, then columns j > i in ascending order, which is the same
set of pairs as j < i in Eq. 13 because b is symmetric.

The paper reports the minimum energy over 50 shots; here a "shot" is an SB
agent, and the best agent is the one of minimum O, ties going to the lowest
agent index.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class _Neumaier:
    """Vectorised compensated accumulator (one lane per agent)."""

    def __init__(self, shape):
        self.s = np.zeros(shape)
        self.c = np.zeros(shape)

    def add(self, v):
        t = self.s + v
        big = np.abs(self.s) >= np.abs(v)
        self.c = self.c + np.where(big, (self.s - t) + v, (v - t) + self.s)
        self.s = t

    def value(self):
        return self.s + self.c


def qubo_energy(a: np.ndarray, b: sp.csr_matrix, T: np.ndarray) -> np.ndarray:
    """O(T) for T of shape [n] (returns a scalar array) or [n, agents]."""
    T = np.asarray(T)
    squeeze = T.ndim == 1
    if squeeze:
        T = T[:, None]
    T = T.astype(np.float64)
    b = sp.csr_matrix(b, dtype=np.float64)
    n, m = T.shape
    acc = _Neumaier(m)
    for i in range(n):
        ti = T[i]
        acc.add(a[i] * ti)
        lo, hi = b.indptr[i], b.indptr[i + 1]
        for p in range(lo, hi):
            j = b.indices[p]
            if j > i:
                acc.add(b.data[p] * (ti * T[j]))
    out = acc.value()
    return out[0] if squeeze else out


def best_agent(energies: np.ndarray) -> int:
    """Index of the minimum energy; the first (lowest index) on ties."""
    return int(np.argmin(np.asarray(energies)))
