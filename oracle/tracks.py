"""Track candidates from a QUBO solution, and efficiency / purity.

Section "QUBO Generation and Track Finding" (last paragraph) and the
Results section (Eq. 18-19).  The paper states the steps but not the
conflict rule or the truth set, so these readings are used:

* selected triplets (T_i = 1) are split into their two doublets; the
  union is the candidate doublet set;
* a doublet (u, v) is dropped if hit u has more than one selected
  outgoing doublet or hit v more than one selected incoming doublet
  (unresolved conflicts);
* the remaining doublets chain into paths; paths with fewer than
  min(4, number of layers) hits are discarded;
* true doublets are hit pairs of one particle on consecutive layers, over
  all particles; TP counts reconstructed doublets that are true, FN true
  doublets not reconstructed, FP reconstructed doublets that are not true.
  Efficiency = TP / (TP + FN), purity = TP / (TP + FP).
"""
from __future__ import annotations

from collections import defaultdict
from typing import List, Optional, Set, Tuple

import numpy as np


def selected_doublets(trip_hits: np.ndarray, T: np.ndarray) -> Set[Tuple[int, int]]:
    out = set()
    for k in np.nonzero(np.asarray(T) != 0)[0]:
        h1, h2, h3 = (int(v) for v in trip_hits[k])
        out.add((h1, h2))
        out.add((h2, h3))
    return out


def resolve_conflicts(dbl: Set[Tuple[int, int]]) -> Set[Tuple[int, int]]:
    n_out = defaultdict(int)
    n_in = defaultdict(int)
    for u, v in dbl:
        n_out[u] += 1
        n_in[v] += 1
    return set((u, v) for (u, v) in dbl if n_out[u] == 1 and n_in[v] == 1)


def chain(dbl: Set[Tuple[int, int]]) -> List[List[int]]:
    """Paths of a graph in which every hit has at most one in and one out edge."""
    nxt = {u: v for u, v in dbl}
    has_in = set(v for _, v in dbl)
    paths = []
    for u in sorted(nxt):
        if u in has_in:
            continue
        path = [u]
        while path[-1] in nxt:
            path.append(nxt[path[-1]])
        paths.append(path)
    return paths


def track_candidates(trip_hits: np.ndarray, T: np.ndarray, min_hits: int) -> List[List[int]]:
    paths = chain(resolve_conflicts(selected_doublets(trip_hits, T)))
    return [p for p in paths if len(p) >= min_hits]


def true_doublets(particle: np.ndarray, layer: np.ndarray,
                  keep_particles: Optional[Set[int]] = None) -> Set[Tuple[int, int]]:
    by_p = defaultdict(list)
    for h, (p, L) in enumerate(zip(particle, layer)):
        if p >= 0 and (keep_particles is None or int(p) in keep_particles):
            by_p[int(p)].append((int(L), h))
    out = set()
    for hits in by_p.values():
        hits.sort()
        for (l1, h1), (l2, h2) in zip(hits, hits[1:]):
            if l2 == l1 + 1:
                out.add((h1, h2))
    return out


def score(candidates: List[List[int]], particle: np.ndarray, layer: np.ndarray,
          keep_particles: Optional[Set[int]] = None):
    """Return (efficiency, purity, TP, FN, FP) over doublets."""
    reco = set()
    for path in candidates:
        for u, v in zip(path, path[1:]):
            reco.add((u, v))
    truth = true_doublets(particle, layer, keep_particles)
    tp = len(reco & truth)
    fn = len(truth - reco)
    fp = len(reco - truth)
    eff = tp / (tp + fn) if tp + fn else 1.0
    pur = tp / (tp + fp) if tp + fp else 1.0
    return eff, pur, tp, fn, fp


def evaluate(ev, trip_hits: np.ndarray, T: np.ndarray):
    """Efficiency / purity of solution T on event `ev` (all particles)."""
    min_hits = min(4, ev.n_layers)
    cands = track_candidates(trip_hits, T, min_hits)
    return score(cands, ev.particle, ev.layer)


def true_triplet_mask(ev, trip_hits: np.ndarray) -> np.ndarray:
    """T_i = 1 iff the three hits of triplet i belong to one particle."""
    p = ev.particle[trip_hits]
    return ((p[:, 0] >= 0) & (p[:, 0] == p[:, 1]) & (p[:, 1] == p[:, 2])).astype(np.int8)
