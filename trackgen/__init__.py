"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates inputs*.  It contains none of the method's
arithmetic (no doublet/triplet/QUBO construction, no Ising mapping, no
simulated-bifurcation step): those live separately in ``oracle/`` (the CPU
reference) and in the HIP library (the product), which share no code.

The events stand in for the barrel-only TrackML events the paper uses
(Dataset section): helical charged particles from the origin in a uniform
2 T solenoid, crossing concentric cylindrical silicon layers, with
r-phi smearing and uniformly distributed noise hits.  No dataset item is
reproduced; every event is drawn from a seeded NumPy PCG64 generator.
"""
from .helix import (EventSpec, Event, generate, RADII_4, RADII_10,
                    SPEED_OF_LIGHT_GEV_PER_T_M)
from .workloads import (WORKLOADS, workload_spec, tiny_spec, plain_spec,
                        precision_spec, stress_spec, batching_specs, STRESS_Z0_MAX)
from .random_qubo import random_qubo

__all__ = [
    "EventSpec", "Event", "generate", "RADII_4", "RADII_10",
    "SPEED_OF_LIGHT_GEV_PER_T_M", "WORKLOADS", "workload_spec", "tiny_spec",
    "plain_spec", "precision_spec", "stress_spec", "batching_specs",
    "random_qubo",
]
