"""Spin relabelling of a triplet QUBO, from its definition.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU baseline use this package.

A relabelling leaves the problem of the section "QUBO formulation"
unchanged: with b' = P b P^T, a' = P a and T' = P T the objective (Eq. 13)
takes the same value.  The order used by the solver sorts triplets by the
azimuth of their middle hit, then by that hit's z, then by index, with the
azimuth compared through the monotone key

    key(x, y) = 1 - x/(|x|+|y|)  for y >= 0,   3 + x/(|x|+|y|)  for y < 0,

(0 at the origin), which equals 0, 1, 2, 3 at phi = 0, pi/2, pi, 3pi/2 and
increases with phi on [0, 2 pi).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def diamond_key(x, y) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = np.abs(x) + np.abs(y)
    with np.errstate(invalid="ignore", divide="ignore"):
        t = np.where(d > 0, x / np.where(d > 0, d, 1.0), 0.0)
    key = np.where(y >= 0, 1.0 - t, 3.0 + t)
    return np.where(d > 0, key, 0.0)


def phi_order(trip_hits: np.ndarray, hit_id: np.ndarray, x: np.ndarray, y: np.ndarray,
              z: np.ndarray) -> np.ndarray:
    """perm[k] = index of the triplet placed at position k."""
    pos = {int(h): k for k, h in enumerate(hit_id)}
    mid = np.array([pos[int(h)] for h in trip_hits[:, 1]], dtype=np.int64)
    key = diamond_key(x[mid], y[mid])
    idx = np.arange(trip_hits.shape[0])
    return np.lexsort((idx, z[mid], key)).astype(np.int32)


def permute(a: np.ndarray, b: sp.csr_matrix, trip_hits: np.ndarray, perm: np.ndarray):
    """(a', b', trip_hits') with spin k of the result = spin perm[k]."""
    perm = np.asarray(perm)
    bp = sp.csr_matrix(b)[perm][:, perm].tocsr()
    bp.sort_indices()
    return a[perm], bp, trip_hits[perm]
