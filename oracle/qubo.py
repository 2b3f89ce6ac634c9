"""QUBO construction from hits: the oracle.

Follows the sections "QUBO Formulation" (Eq. 13-15) and "QUBO Generation
and Track Finding" (Eq. 16-17 and the five-hit rule) of the paper.  Written
as a straight sequence of the paper's steps over plain arrays and Python
containers; speed is not a goal.

Readings taken where the paper is silent or garbled (each one is a parameter
where that makes sense):

* Doublets join hits on adjacent layers with |dphi| < 0.1 rad.  The paper
  delegates doublet seeding to an external trigger code; the window is the
  workload's.  The decision is libm-free: dot > 0 and |cross| < tan(0.1) dot
  with tan(0.1) one shared FP64 literal.  An optional |z0| cut is off.
* The curvature in Eq. 16/17 is the signed transverse curvature
  kappa = 1/R in mm^-1 (Menger curvature of the three hits); read in GeV^-1
  the printed cut would keep only pT above 1.25 TeV.
* delta-theta of a triplet is the angle between the (dr, dz) directions of
  its two doublets; the cut decision uses a cross/dot test against the
  tan(0.1) literal, the value (needed by Eq. 14) uses atan2.
* Holes H = (last layer - first layer - 2); with adjacent-layer doublets it
  is always 0.
* Eq. 14 sums kappa (mm^-1) and delta-theta (rad) unnormalised.
* Eq. 15 is printed with a positive exponent, which would make a_i negative
  and unbounded; the reading used is a_i = alpha (1 - exp(-|d0|/gamma)) +
  beta (1 - exp(-|z0|/lambda)) with d0, z0 in mm, a penalty in [0, alpha+beta).
* The five-hit rule keeps an Eq.-17-passing quadruplet (i -> j) if some
  passing quadruplet (j -> k) or (k -> i) exists (one pass), with the hit
  requirement min(5, number of layers) so that it is vacuous on a 4-layer
  barrel.  Triplets in no kept quadruplet are dropped.
* b_ij (Eq. 13): -S_ij for kept quadruplets; +1 when two triplets share a
  hit and are not shifted windows of one hit chain; 0 otherwise (no shared
  hit, a consistent shift by two, or a shift by one that is not a kept
  quadruplet).

Every arithmetic expression that decides membership is written in one fixed
order of IEEE +, -, *, /, sqrt (no libm, no fused multiply-add), so an
independent implementation evaluating the same expressions takes the same
decisions bit for bit.
"""
from __future__ import annotations

import dataclasses
import math
from collections import defaultdict
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

# tan(0.1) rounded to FP64; the shared literal of every angle-window test.
TAN_0P1 = 0.10033467208545055


@dataclasses.dataclass(frozen=True)
class BuildParams:
    dphi_tan: float = TAN_0P1     # doublet window, as tan(dphi_max)
    z0_max: float = 0.0           # <= 0: no doublet z0 cut
    curv_max: float = 8e-4        # Eq. 16, |kappa| in mm^-1
    dtheta_tan: float = TAN_0P1   # Eq. 16, tan(dtheta_max)
    max_holes: int = 1            # Eq. 16
    dcurv_max: float = 1e-4       # Eq. 17
    s_min: float = 0.2            # Eq. 17
    min_track_hits: int = -1      # five-hit rule; -1: min(5, n_layers)
    alpha: float = 0.5            # Eq. 15
    beta: float = 0.2
    gamma: float = 1.0
    lam: float = 0.5


@dataclasses.dataclass
class Qubo:
    n: int
    a: np.ndarray                 # float64 [n]
    b: sp.csr_matrix              # float64 [n, n], symmetric, zero diagonal
    trip_hits: np.ndarray         # int64 [n, 3], canonical order
    # diagnostics (not part of the QUBO itself)
    doublets: np.ndarray          # int64 [nd, 2] all doublets (before pruning)
    triplets_all: np.ndarray      # int64 [nt, 3] Eq.16-passing triplets
    quads_pass: np.ndarray        # int64 [nq, 2] Eq.17-passing (i, j) in triplets_all ids
    quads_kept: np.ndarray        # int64 [nk, 2] kept after the five-hit rule
    kappa: np.ndarray             # float64 [n]
    dtheta: np.ndarray            # float64 [n]
    d0: np.ndarray                # float64 [n]
    z0: np.ndarray                # float64 [n]


def _radius(x, y):
    return math.sqrt(x * x + y * y)


def find_doublets(x, y, z, layer, p: BuildParams) -> np.ndarray:
    """Adjacent-layer hit pairs inside the azimuthal window, ordered by
    (id1, id2).  Hit ids are array indices."""
    n_layers = int(layer.max()) + 1 if layer.size else 0
    out = []
    for L in range(n_layers - 1):
        ia = np.nonzero(layer == L)[0]
        ib = np.nonzero(layer == L + 1)[0]
        if ia.size == 0 or ib.size == 0:
            continue
        for s in range(0, ia.size, 256):
            a = ia[s:s + 256]
            x1 = x[a][:, None]
            y1 = y[a][:, None]
            x2 = x[ib][None, :]
            y2 = y[ib][None, :]
            cross = x1 * y2 - y1 * x2
            dot = x1 * x2 + y1 * y2
            ok = (dot > 0.0) & (np.abs(cross) < p.dphi_tan * dot)
            if p.z0_max > 0.0:
                r1 = np.sqrt(x1 * x1 + y1 * y1)
                r2 = np.sqrt(x2 * x2 + y2 * y2)
                z1 = z[a][:, None]
                z2 = z[ib][None, :]
                z0 = z1 - r1 * (z2 - z1) / (r2 - r1)
                ok &= np.abs(z0) <= p.z0_max
            r, c = np.nonzero(ok)
            out.append(np.stack([a[r], ib[c]], axis=1))
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    d = np.concatenate(out).astype(np.int64)
    order = np.lexsort((d[:, 1], d[:, 0]))
    return d[order]


def triplet_features(x, y, z, layer, h1, h2, h3):
    """Geometry of one hit triplet, in the fixed evaluation order.

    Returns (kappa, theta_ok_cross, theta_dot, holes, d0, z0)."""
    x1, y1, z1 = x[h1], y[h1], z[h1]
    x2, y2, z2 = x[h2], y[h2], z[h2]
    x3, y3, z3 = x[h3], y[h3], z[h3]
    ux = x2 - x1
    uy = y2 - y1
    vx = x3 - x2
    vy = y3 - y2
    wx = x3 - x1
    wy = y3 - y1
    cr = ux * vy - uy * vx
    nu = math.sqrt(ux * ux + uy * uy)
    nv = math.sqrt(vx * vx + vy * vy)
    nw = math.sqrt(wx * wx + wy * wy)
    kappa = (2.0 * cr) / ((nu * nv) * nw)
    r1 = _radius(x1, y1)
    r2 = _radius(x2, y2)
    r3 = _radius(x3, y3)
    d1r = r2 - r1
    d1z = z2 - z1
    d2r = r3 - r2
    d2z = z3 - z2
    tcross = d1r * d2z - d1z * d2r
    tdot = d1r * d2r + d1z * d2z
    holes = int(layer[h3]) - int(layer[h1]) - 2
    # transverse impact parameter from the circle through the three hits,
    # centre found relative to the first hit
    bb = ux * ux + uy * uy
    cc = wx * wx + wy * wy
    den = 2.0 * (ux * wy - uy * wx)
    if den != 0.0:
        ocx = (wy * bb - uy * cc) / den
        ocy = (ux * cc - wx * bb) / den
        xc = x1 + ocx
        yc = y1 + ocy
        rad = math.sqrt(ocx * ocx + ocy * ocy)
        d0 = abs(math.sqrt(xc * xc + yc * yc) - rad)
    else:  # collinear: distance of the line to the origin
        d0 = abs(x1 * wy - y1 * wx) / nw
    z0 = z1 - r1 * d1z / d1r
    return kappa, tcross, tdot, holes, d0, z0


def quad_strength(dk: float, dtheta_i: float, dtheta_j: float,
                  holes_i: float, holes_j: float) -> float:
    """S_ij of Eq. 14 from |delta kappa|, the two delta-thetas and holes."""
    hsum = 1.0 + holes_i + holes_j
    return (1.0 - 0.5 * (dk + max(dtheta_i, dtheta_j))) / (hsum * hsum)


def bias_weight(d0: float, z0: float, p: BuildParams) -> float:
    """a_i of Eq. 15 (decaying-exponential reading)."""
    return (p.alpha * (1.0 - math.exp(-abs(d0) / p.gamma))
            + p.beta * (1.0 - math.exp(-abs(z0) / p.lam)))


def classify_pair(tu, tv) -> str:
    """Relation of two distinct triplets (hit-id tuples in layer order):
    'none' (no shared hit), 'shift1' (consecutive windows of one chain,
    sharing two hits), 'shift2' (windows sharing one end hit) or
    'conflict' (any other shared hit)."""
    if not (set(tu) & set(tv)):
        return "none"
    if tuple(tu[1:]) == tuple(tv[:2]) or tuple(tv[1:]) == tuple(tu[:2]):
        return "shift1"
    if tu[2] == tv[0] or tv[2] == tu[0]:
        return "shift2"
    return "conflict"


def build(x, y, z, layer, p: BuildParams = BuildParams()) -> Qubo:
    """Hits -> QUBO (a, b), following the paper's construction steps."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    layer = np.asarray(layer, dtype=np.int64)
    n_layers = int(layer.max()) + 1 if layer.size else 0
    mth = p.min_track_hits if p.min_track_hits >= 0 else min(5, n_layers)
    if mth > 5:
        raise ValueError("five-hit rule implemented for min_track_hits <= 5")

    # 1. doublets
    dbl = find_doublets(x, y, z, layer, p)

    # 2. triplets: join (h1,h2) with (h2,h3) on the shared middle hit; Eq. 16
    outgoing: Dict[int, List[int]] = defaultdict(list)
    for h1, h2 in dbl:
        outgoing[int(h1)].append(int(h2))
    trips: List[Tuple[int, int, int]] = []
    feats = []
    for h1, h2 in dbl:
        h1 = int(h1)
        h2 = int(h2)
        for h3 in outgoing.get(h2, ()):
            kap, tc, td, holes, d0, z0 = triplet_features(x, y, z, layer, h1, h2, h3)
            if holes > p.max_holes:
                continue
            if not (abs(kap) <= p.curv_max):
                continue
            if not (td > 0.0 and abs(tc) <= p.dtheta_tan * td):
                continue
            dth = math.atan2(abs(tc), td)
            trips.append((h1, h2, h3))
            feats.append((kap, dth, float(holes), d0, z0))
    # (dbl is sorted by (h1, h2) and each outgoing list ascends in h3, so
    #  trips is already in (h1, h2, h3) order)

    # 3. quadruplets: (h1,h2,h3) -> (h2,h3,h4), joined on the pair (h2,h3); Eq. 14, 17
    by_first_pair: Dict[Tuple[int, int], List[int]] = defaultdict(list)
    for t, (h1, h2, h3) in enumerate(trips):
        by_first_pair[(h1, h2)].append(t)
    quads = []
    s_val = {}
    for i, (h1, h2, h3) in enumerate(trips):
        ki, dthi, hi = feats[i][0], feats[i][1], feats[i][2]
        for j in by_first_pair.get((h2, h3), ()):
            kj, dthj, hj = feats[j][0], feats[j][1], feats[j][2]
            dk = abs(ki - kj)
            if not (dk <= p.dcurv_max):
                continue
            s = quad_strength(dk, dthi, dthj, hi, hj)
            if not (s > p.s_min):
                continue
            quads.append((i, j))
            s_val[(i, j)] = s

    # 4. five-hit rule (one pass over the Eq.-17-passing set)
    if mth >= 5:
        has_out = set(i for i, _ in quads)
        has_in = set(j for _, j in quads)
        kept = [(i, j) for (i, j) in quads if (j in has_out) or (i in has_in)]
    else:
        kept = list(quads)

    # 5. prune triplets in no kept quadruplet; canonical (h1,h2,h3) order
    alive = sorted(set(t for q in kept for t in q), key=lambda t: trips[t])
    new_id = {t: k for k, t in enumerate(alive)}
    n = len(alive)
    trip_hits = np.array([trips[t] for t in alive], dtype=np.int64).reshape(n, 3)

    # 6. bias weights, Eq. 15 (sign reading: decaying exponentials)
    a = np.zeros(n, dtype=np.float64)
    kappa = np.zeros(n)
    dtheta = np.zeros(n)
    d0s = np.zeros(n)
    z0s = np.zeros(n)
    for k, t in enumerate(alive):
        kap, dth, _, d0, z0 = feats[t]
        kappa[k], dtheta[k], d0s[k], z0s[k] = kap, dth, d0, z0
        a[k] = bias_weight(d0, z0, p)

    # 7. couplings b_ij, Eq. 13
    coup: Dict[Tuple[int, int], float] = {}
    for (i, j) in kept:
        u, v = new_id[i], new_id[j]
        coup[(min(u, v), max(u, v))] = -s_val[(i, j)]
    by_hit: Dict[int, List[int]] = defaultdict(list)
    for k in range(n):
        for h in trip_hits[k]:
            by_hit[int(h)].append(k)
    for members in by_hit.values():
        for ai in range(len(members)):
            for bi in range(ai + 1, len(members)):
                u, v = members[ai], members[bi]
                key = (min(u, v), max(u, v))
                if key in coup:
                    continue
                rel = classify_pair(tuple(trip_hits[u]), tuple(trip_hits[v]))
                if rel == "conflict":
                    coup[key] = 1.0
                # 'shift1' without a kept quadruplet and 'shift2' couple with 0
    rows, cols, vals = [], [], []
    for (u, v), w in coup.items():
        rows += [u, v]
        cols += [v, u]
        vals += [w, w]
    b = sp.csr_matrix((np.array(vals, dtype=np.float64),
                       (np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64))),
                      shape=(n, n))
    b.sort_indices()

    qa = np.array(quads, dtype=np.int64).reshape(-1, 2)
    qk = np.array(kept, dtype=np.int64).reshape(-1, 2)
    return Qubo(n=n, a=a, b=b, trip_hits=trip_hits, doublets=dbl,
                triplets_all=np.array(trips, dtype=np.int64).reshape(-1, 3),
                quads_pass=qa, quads_kept=qk, kappa=kappa, dtheta=dtheta,
                d0=d0s, z0=z0s)


def build_event(ev, p: BuildParams = BuildParams()) -> Qubo:
    return build(ev.x, ev.y, ev.z, ev.layer, p)
