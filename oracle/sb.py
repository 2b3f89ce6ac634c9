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
* the result is the final state of every agent (readout s = sgn(x));
* time-to-target needs the energies reached along the way: at every
  `ckpt_every`-th step (after steps ckpt_every, 2 ckpt_every, ... <= K) the
  state is read out, T = (1 + sgn x)/2, and its FP64 objective O(T) of
  Eq. 13 recorded per agent; the best-so-far trace is the running minimum
  over agents and checkpoints.

State arrays are [n, agents]; every agent is an independent shot.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import energy as _energy
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
    agent_trace: Optional[np.ndarray] = None  # [n_ckpt, agents] O(T) at each checkpoint
    trace: Optional[np.ndarray] = None        # [n_ckpt] best-so-far over agents
    readout_margin: Optional[np.ndarray] = None  # per agent: min |x| at checkpoint readouts


def run(J: sp.csr_matrix, h: np.ndarray, c0: float, mode: str, agents: int,
        steps: int, dt: float = 1.0, a0: float = 1.0, seed: int = 0,
        event: int = 0, x0: Optional[np.ndarray] = None,
        y0: Optional[np.ndarray] = None, margin_steps: int = 0,
        ckpt_every: int = 0, qubo=None) -> SBResult:
    """Integrate `steps` symplectic-Euler steps for `agents` shots.

    `margin_steps` > 0 records decision margins over the first that many
    steps (used to tell a legitimate FP32 divergence from a wrong result).
    `ckpt_every` > 0 with `qubo` = (a, b) of Eq. 13 records the readout
    energies after every ckpt_every-th step (steps // ckpt_every
    checkpoints)."""
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
    n_ckpt = steps // ckpt_every if ckpt_every > 0 else 0
    if n_ckpt and qubo is None:
        raise ValueError("checkpoint energies need qubo = (a, b)")
    agent_trace = np.zeros((n_ckpt, agents))
    readout_margin = np.full(agents, np.inf)

    def checkpoint(done):
        # `done` steps have been taken; record every ckpt_every-th
        nonlocal readout_margin
        if n_ckpt and done % ckpt_every == 0 and done // ckpt_every <= n_ckpt:
            agent_trace[done // ckpt_every - 1] = _energy.qubo_energy(qubo[0], qubo[1],
                                                                      readout(x))
            readout_margin = np.minimum(readout_margin, np.abs(x).min(axis=0))

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
            checkpoint(k + 1)
            continue
        y = y + dt * (c0 * F - (a0 - a_k) * x)
        x = x + dt * a0 * y
        if k < margin_steps:
            wall_margin = np.minimum(wall_margin, np.abs(np.abs(x) - 1.0).min(axis=0))
        hit = np.abs(x) > 1.0
        x = np.where(hit, sgn(x), x)
        y = np.where(hit, 0.0, y)
        checkpoint(k + 1)
    sign_margin = np.minimum(sign_margin, np.abs(x).min(axis=0))
    trace = np.minimum.accumulate(agent_trace.min(axis=1)) if n_ckpt else None
    return SBResult(x=x, y=y, sign_margin=sign_margin, wall_margin=wall_margin,
                    agent_trace=agent_trace if n_ckpt else None, trace=trace,
                    readout_margin=readout_margin if n_ckpt else None)


def readout(x: np.ndarray) -> np.ndarray:
    """Binary QUBO variables T = (1 + sgn(x)) / 2 as int8, same shape as x."""
    return (x >= 0.0).astype(np.int8)
