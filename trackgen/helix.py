"""Helix-in-solenoid event generator (input side only).

Geometry follows the paper's Dataset section: a barrel of concentric
cylindrical layers inside a 2 T solenoid, barrel hits only.  A particle of
charge q, transverse momentum pT [GeV], pseudorapidity eta and initial
azimuth phi0 leaves the origin on a helix whose transverse projection is a
circle of radius R = pT / (0.299792458 * B) metres through the origin.  At a
layer of radius r it is found at

    alpha = asin(r / 2R),   phi = phi0 - q * alpha,   z = 2 R alpha sinh(eta)

(transverse arc length 2 R alpha times dz/ds_T = sinh(eta)).  A hit exists if
r < 2R and |z| <= z_half of that layer.  The azimuth is smeared by a Gaussian
of width sigma_rphi / r; z is not smeared.  Noise hits are added per layer,
round(noise_frac * true hits on that layer) of them, uniform in phi and z.

Hits are returned sorted by (layer, phi in [0, 2pi)); a hit's id is its rank
in that order.  Downstream code uses only (x, y, z, layer) of a hit; the
particle id (-1 for noise) is truth used for scoring.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

SPEED_OF_LIGHT_GEV_PER_T_M = 0.299792458  # pT[GeV] = 0.2998 * B[T] * R[m]

RADII_10 = (32.0, 72.0, 116.0, 172.0, 260.0, 360.0, 500.0, 660.0, 820.0, 1020.0)
RADII_4 = (32.0, 72.0, 116.0, 172.0)


@dataclasses.dataclass(frozen=True)
class EventSpec:
    """Recipe of one synthetic event (all lengths in mm, momenta in GeV)."""
    n_particles: int
    pt_min: float = 0.5
    pt_max: float = 20.0
    eta_max: float = 1.5
    noise_frac: float = 0.10
    radii: Tuple[float, ...] = RADII_10
    z_half: Optional[Tuple[float, ...]] = None  # None: max(400, 1.1 r sinh(eta_max))
    b_field: float = 2.0
    sigma_rphi: float = 0.020

    def layer_z_half(self) -> Tuple[float, ...]:
        if self.z_half is not None:
            return tuple(float(v) for v in self.z_half)
        s = math.sinh(self.eta_max)
        return tuple(max(400.0, r * s * 1.1) for r in self.radii)


@dataclasses.dataclass
class Event:
    """Hits (sorted by layer, phi) plus the particle table used to make them."""
    x: np.ndarray          # float64 [n_hits] mm
    y: np.ndarray          # float64 [n_hits] mm
    z: np.ndarray          # float64 [n_hits] mm
    layer: np.ndarray      # int32   [n_hits] 0 = innermost
    particle: np.ndarray   # int64   [n_hits] particle index, -1 = noise
    hit_id: np.ndarray     # int64   [n_hits] == arange(n_hits)
    q: np.ndarray          # int32   [n_particles] charge +-1
    pt: np.ndarray         # float64 [n_particles] GeV
    eta: np.ndarray        # float64 [n_particles]
    phi0: np.ndarray       # float64 [n_particles]
    spec: EventSpec
    seed: int

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_layers(self) -> int:
        return len(self.spec.radii)

    def radius_of_curvature(self) -> np.ndarray:
        """Transverse radius R [mm] of every particle's helix."""
        return self.pt / (SPEED_OF_LIGHT_GEV_PER_T_M * self.spec.b_field) * 1000.0

    def hits_struct(self) -> np.ndarray:
        """Hits as a packed record array matching the C ``sbt_hit`` layout
        {int64 hit_id; int32 layer; int32 pad; double x, y, z}."""
        dt = np.dtype([("hit_id", "<i8"), ("layer", "<i4"), ("pad", "<i4"),
                       ("x", "<f8"), ("y", "<f8"), ("z", "<f8")])
        out = np.zeros(self.n_hits, dtype=dt)
        out["hit_id"] = self.hit_id
        out["layer"] = self.layer
        out["x"] = self.x
        out["y"] = self.y
        out["z"] = self.z
        return out


def generate(spec: EventSpec, seed: int) -> Event:
    """Draw one event.  The draw order is fixed so that a seed names an event."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(spec.n_particles)
    n_layers = len(spec.radii)
    radii = np.asarray(spec.radii, dtype=np.float64)
    z_half = np.asarray(spec.layer_z_half(), dtype=np.float64)

    q = np.where(rng.random(n) < 0.5, -1, 1).astype(np.int32)
    pt = np.exp(rng.uniform(math.log(spec.pt_min), math.log(spec.pt_max), n))
    eta = rng.uniform(-spec.eta_max, spec.eta_max, n)
    phi0 = rng.uniform(0.0, 2.0 * math.pi, n)
    smear = rng.standard_normal((n, n_layers))

    big_r = pt / (SPEED_OF_LIGHT_GEV_PER_T_M * spec.b_field) * 1000.0  # mm

    hx, hy, hz, hl, hp = [], [], [], [], []
    n_true = np.zeros(n_layers, dtype=np.int64)
    for li in range(n_layers):
        r = radii[li]
        reach = r < 2.0 * big_r
        ratio = np.where(reach, r / (2.0 * big_r), 0.0)
        alpha = np.arcsin(ratio)
        s = 2.0 * big_r * alpha
        z = s * np.sinh(eta)
        ok = reach & (np.abs(z) <= z_half[li])
        phi = phi0 - q * alpha + smear[:, li] * (spec.sigma_rphi / r)
        idx = np.nonzero(ok)[0]
        n_true[li] = idx.size
        hx.append(r * np.cos(phi[idx]))
        hy.append(r * np.sin(phi[idx]))
        hz.append(z[idx])
        hl.append(np.full(idx.size, li, dtype=np.int32))
        hp.append(idx.astype(np.int64))

    for li in range(n_layers):
        r = radii[li]
        cnt = int(round(spec.noise_frac * n_true[li]))
        phi = rng.uniform(0.0, 2.0 * math.pi, cnt)
        z = rng.uniform(-z_half[li], z_half[li], cnt)
        hx.append(r * np.cos(phi))
        hy.append(r * np.sin(phi))
        hz.append(z)
        hl.append(np.full(cnt, li, dtype=np.int32))
        hp.append(np.full(cnt, -1, dtype=np.int64))

    x = np.concatenate(hx)
    y = np.concatenate(hy)
    z = np.concatenate(hz)
    layer = np.concatenate(hl)
    particle = np.concatenate(hp)
    phi_sort = np.mod(np.arctan2(y, x), 2.0 * math.pi)
    order = np.lexsort((phi_sort, layer))
    return Event(x=x[order].copy(), y=y[order].copy(), z=z[order].copy(),
                 layer=layer[order].copy(), particle=particle[order].copy(),
                 hit_id=np.arange(x.size, dtype=np.int64),
                 q=q, pt=pt, eta=eta, phi0=phi0, spec=spec, seed=int(seed))
