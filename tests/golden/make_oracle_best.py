"""Write oracle_best_plain.json: the FP64 oracle's best QUBO energy on the
benchmarked event (200 particles, seed 100; 256 agents, 5000 steps, solver
seed 0) for bSB and dSB.  The time-to-target measurement uses
E* + 0.5 |E*| as its target.  Calls only ``oracle`` and ``trackgen``.

    python tests/golden/make_oracle_best.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import trackgen as tg  # noqa: E402
from oracle import energy, ising, qubo, sb  # noqa: E402

EVENT_SEED, AGENTS, STEPS, SOLVER_SEED = 100, 256, 5000, 0


def main():
    ev = tg.generate(tg.plain_spec(), EVENT_SEED)
    q = qubo.build_event(ev)
    isg = ising.from_qubo(q.a, q.b)
    out = {"event": "plain", "event_seed": EVENT_SEED, "n": q.n, "nnz": int(q.b.nnz),
           "agents": AGENTS, "steps": STEPS, "solver_seed": SOLVER_SEED, "modes": {}}
    for mode in ("bsb", "dsb"):
        t = time.time()
        r = sb.run(isg.J, isg.h, isg.c0, mode, AGENTS, STEPS, seed=SOLVER_SEED)
        E = energy.qubo_energy(q.a, q.b, sb.readout(r.x))
        out["modes"][mode] = {"best": float(E.min()), "best_agent": int(np.argmin(E)),
                              "mean": float(E.mean()), "worst": float(E.max()),
                              "oracle_seconds": round(time.time() - t, 2)}
        print(mode, out["modes"][mode], flush=True)
    with open(os.path.join(HERE, "oracle_best_plain.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
