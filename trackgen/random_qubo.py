"""Seeded random QUBO instances with the value structure of the track QUBO.

Linear weights a_i in [0, 0.7) (the range of the bias weight), couplings
b_ij = +1 (conflict) or -S with S in (0.2, 1] (quadruplet reward), on a random
symmetric sparsity pattern.  Returned as dense FP64 arrays; callers convert
to whatever storage they need.  Used for brute-force and solver tests on
small N where no detector geometry is needed.
"""
from __future__ import annotations

import numpy as np


def random_qubo(n: int, seed: int, density: float = 0.3,
                conflict_frac: float = 0.6):
    """Return (a[n], b[n, n]) with b symmetric and zero on the diagonal."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.0, 0.7, n)
    b = np.zeros((n, n), dtype=np.float64)
    iu, ju = np.triu_indices(n, 1)
    present = rng.random(iu.size) < density
    conflict = rng.random(iu.size) < conflict_frac
    strength = rng.uniform(0.2, 1.0, iu.size)
    vals = np.where(conflict, 1.0, -strength)
    vals = np.where(present, vals, 0.0)
    b[iu, ju] = vals
    b[ju, iu] = vals
    return a, b
