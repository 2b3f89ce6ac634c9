"""The five synthetic workloads (event recipes plus solver settings).

Each entry names an event recipe, the event seeds, the SB form and the
(agents, steps) of the solve.  The sizes are the ones the benchmark and the
full-size tests run; N (number of triplets) and nnz are measured, not set.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Tuple

import numpy as np

from .helix import EventSpec, RADII_4, RADII_10


def tiny_spec() -> EventSpec:
    """4-layer barrel, |z| < 400 mm, 10 particles of 1-10 GeV, |eta| < 1, no noise."""
    return EventSpec(n_particles=10, pt_min=1.0, pt_max=10.0, eta_max=1.0,
                     noise_frac=0.0, radii=RADII_4, z_half=(400.0,) * 4)


def plain_spec(n_particles: int = 200) -> EventSpec:
    """10-layer barrel, pT 0.5-20 GeV, |eta| < 1.5, +10% noise hits."""
    return EventSpec(n_particles=n_particles, pt_min=0.5, pt_max=20.0,
                     eta_max=1.5, noise_frac=0.10, radii=RADII_10)


def precision_spec() -> EventSpec:
    return plain_spec(1000)


def stress_spec() -> EventSpec:
    """5000 particles, |eta| < 2, +20% noise."""
    return EventSpec(n_particles=5000, pt_min=0.5, pt_max=20.0, eta_max=2.0,
                     noise_frac=0.20, radii=RADII_10)


# The stress event keeps only doublets whose straight-line extrapolation to
# the beam axis lands within |z0| <= 300 mm (the luminous region's extent
# with margin): without that cut the doublet combinatorics of 5000
# particles plus noise give far more than the ~2e5 triplets of the workload.
STRESS_Z0_MAX = 300.0


def batching_specs(n_events: int = 512, count_seed: int = 999,
                   first_event_seed: int = 1000) -> List[Tuple[EventSpec, int]]:
    """512 events whose particle counts are 20 + floor(981 U), U from seed 999."""
    rng = np.random.Generator(np.random.PCG64(count_seed))
    counts = 20 + np.floor(981.0 * rng.random(n_events)).astype(np.int64)
    return [(plain_spec(int(c)), first_event_seed + k) for k, c in enumerate(counts)]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    spec: EventSpec
    seeds: Tuple[int, ...]
    modes: Tuple[str, ...]     # "bsb" / "dsb"
    agents: int
    steps: int
    storage: str               # J storage the workload is specified with
    z0_max: float = 0.0        # doublet |z0| cut of the QUBO build (0: off)


WORKLOADS: Dict[str, Workload] = {
    "tiny": Workload("tiny", tiny_spec(), tuple(range(1, 11)), ("dsb",), 32, 2000,
                     "csr-fp32"),
    "plain": Workload("plain", plain_spec(), tuple(range(100, 105)), ("bsb", "dsb"),
                      256, 5000, "csr-fp32"),
    "precision": Workload("precision", precision_spec(), (200, 201, 202), ("dsb",),
                          1024, 5000, "csr-bf16"),
    "stress": Workload("stress", stress_spec(), (300,), ("bsb",), 512, 10000,
                       "csr-fp8", STRESS_Z0_MAX),
}


def workload_spec(name: str) -> Workload:
    return WORKLOADS[name]
