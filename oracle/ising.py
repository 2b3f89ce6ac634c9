"""QUBO -> Ising map and the SB coupling scale c0.

The paper states the problem as the QUBO of Eq. 13 over T in {0, 1} and
reports "Ising energies" (Results section) without printing the map.  With
T = (1 + s)/2, s in {-1, +1} and b symmetric with zero diagonal,

    O(T) = C - 1/2 s^T J s - h^T s

where  J = -b/4,   h_i = -(a_i/2 + 1/4 sum_j b_ij),
       C = sum_i a_i/2 + sum_{i<j} b_ij/4.

SB minimises E(s) = -1/2 s^T J s - h^T s; the field h enters the force as
F = J x + h (the exact gradient of 1/2 x^T J x + h^T x), since Eq. 2/6/10
are written for a field-free Ising model.

c0 (the paper keeps it fixed without printing it) is read as
c0 = 0.5 / (sqrt(N) sigma_J), sigma_J the population standard deviation of
all N^2 entries of J, zeros included.  If sigma_J is 0 the couplings vanish
and c0 = 0.5 / sqrt(N) is used (a reading: only the field then acts).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Ising:
    n: int
    J: sp.csr_matrix      # float64, symmetric, zero diagonal
    h: np.ndarray         # float64 [n]
    C: float              # O(T) = E_ising(s) + C
    c0: float


def from_qubo(a: np.ndarray, b: sp.csr_matrix) -> Ising:
    n = int(a.shape[0])
    b = sp.csr_matrix(b, dtype=np.float64)
    J = (-0.25 * b).tocsr()
    J.sort_indices()
    rowsum_b = np.asarray(b.sum(axis=1)).ravel()
    h = -(0.5 * a + 0.25 * rowsum_b)
    upper = sp.triu(b, k=1)
    C = 0.5 * float(np.sum(a)) + 0.25 * float(upper.sum())
    return Ising(n=n, J=J, h=h, C=C, c0=coupling_scale(J, n))


def coupling_scale(J: sp.csr_matrix, n: int) -> float:
    """c0 = 0.5 / (sqrt(N) * population std of the N^2 entries of J)."""
    if n <= 0:
        raise ValueError("empty problem")
    n2 = float(n) * float(n)
    s1 = float(J.data.sum())
    s2 = float(np.dot(J.data, J.data))
    var = s2 / n2 - (s1 / n2) ** 2
    sigma = math.sqrt(var) if var > 0.0 else 0.0
    if sigma == 0.0:
        return 0.5 / math.sqrt(n)
    return 0.5 / (math.sqrt(n) * sigma)


def ising_energy(ising: Ising, s: np.ndarray) -> np.ndarray:
    """E(s) = -1/2 s^T J s - h^T s for s of shape [n] or [n, agents]."""
    s = np.asarray(s, dtype=np.float64)
    Js = ising.J @ s
    return -0.5 * np.sum(s * Js, axis=0) - ising.h @ s
