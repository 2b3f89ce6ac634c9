"""Ballistic and discrete simulated bifurcation, FP64, step by step.

Section "Simulated Bifurcation" of the paper:

* bSB, Eq. 5-8:  dx_i/dt = a0 y_i,
                 dy_i/dt = -(a0 - a(t)) x_i + c0 sum_j J_ij x_j,
  with perfectly inelastic walls at |x_i| > 1: x_i <- sgn(x_i), y_i <- 0.
* dSB, Eq. 9-12: the same, with x_j replaced by sgn(x_j) in the coupling.
* aSB, Eq. 1-4: dy_i/dt = -(x_i^2 + a0 - a(t)) x_i + c0 sum_j J_ij x_j, no
  walls (the quartic term of V_aSB bounds the motion).
* a(t) rises monotonically from zero; a0, dt = 1 and c0 fixed (Results).
* integration by the symplectic Euler method; all spins update at once.

Readings (the paper does not print these):
* schedule a_k = a0 * k / K for k = 0 .. K-1 (linear ramp);
* step order: kick y with the old x, drift x with the new y, then walls;
* the Ising field enters the force: F = J x + h (bSB), J sgn(x) + h (dSB);
* sgn(0) = +1; the wall test is strict, |x| > 1;
* start from the Philox draw of ``philox.initial_state``;
* the result is the final state of every agent (readout s = sgn(x)).

State arrays are [n, agents]; every agent is an independent shot.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

from .philox import initial_state

BSB = "bsb"
DSB = "dsb"
ASB = "asb"


def sgn(x: np.ndarray) -> np.ndarray:
    """Sign with sgn(0) = +1."""
    return np.where(x >= 0.0, 1.0, -1.0)


@dataclasses.dataclass
class SBResult:
    x: np.ndarray                # final positions [n, agents]
    y: np.ndarray                # final momenta   [n, agents]
    sign_margin: np.ndarray      # per agent: min |x| where sgn(x) was used (dSB) or read out
    wall_margin: np.ndarray      # per agent: min ||x| - 1| at wall tests


def run(J: sp.csr_matrix, h: np.ndarray, c0: float, mode: str, agents: int,
        steps: int, dt: float = 1.0, a0: float = 1.0, seed: int = 0,
        event: int = 0, x0: Optional[np.ndarray] = None,
        y0: Optional[np.ndarray] = None, margin_steps: int = 0) -> SBResult:
    """Integrate `steps` symplectic-Euler steps for `agents` shots.

    `margin_steps` > 0 records decision margins over the first that many
    steps (used to tell a legitimate FP32 divergence from a wrong result)."""
    if mode not in (BSB, DSB, ASB):
        raise ValueError(mode)
    n = int(h.shape[0])
    J = sp.csr_matrix(J, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    if x0 is None or y0 is None:
        x, y = initial_state(n, agents, seed, event)
    else:
        x = np.array(x0, dtype=np.float64, copy=True)
        y = np.array(y0, dtype=np.float64, copy=True)
    sign_margin = np.full(agents, np.inf)
    wall_margin = np.full(agents, np.inf)
    hcol = h[:, None]
    for k in range(steps):
        a_k = a0 * k / steps
        if mode == DSB:
            F = J @ sgn(x) + hcol
            if k < margin_steps:
                sign_margin = np.minimum(sign_margin, np.abs(x).min(axis=0))
        else:
            F = J @ x + hcol
        if mode == ASB:
            y = y + dt * (c0 * F - (x * x + (a0 - a_k)) * x)
            x = x + dt * a0 * y
            continue
        y = y + dt * (c0 * F - (a0 - a_k) * x)
        x = x + dt * a0 * y
        if k < margin_steps:
            wall_margin = np.minimum(wall_margin, np.abs(np.abs(x) - 1.0).min(axis=0))
        hit = np.abs(x) > 1.0
        x = np.where(hit, sgn(x), x)
        y = np.where(hit, 0.0, y)
    sign_margin = np.minimum(sign_margin, np.abs(x).min(axis=0))
    return SBResult(x=x, y=y, sign_margin=sign_margin, wall_margin=wall_margin)


def readout(x: np.ndarray) -> np.ndarray:
    """Binary QUBO variables T = (1 + sgn(x)) / 2 as int8, same shape as x."""
    return (x >= 0.0).astype(np.int8)
