"""Write the FP64 oracle's best QUBO energies used as time-to-target
references.  Calls only ``oracle`` and ``trackgen``.

* oracle_best_plain.json: 200 particles, event seed 100; 256 agents,
  5000 steps, solver seed 0; bSB and dSB.
* oracle_best_precision.json: 1000 particles, event seed 200; dSB, 5000
  steps, solver seed 0, agents 0..31 only (agents are independent, so this
  is the oracle's best over the first 32 of the 1024 agents the precision
  workload runs).

    python tests/golden/make_oracle_best.py [plain|precision]
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


def precision():
    ev = tg.generate(tg.precision_spec(), 200)
    q = qubo.build_event(ev)
    isg = ising.from_qubo(q.a, q.b)
    out = {"event": "precision", "event_seed": 200, "n": q.n, "nnz": int(q.b.nnz),
           "agents": 32, "agents_of_workload": 1024, "steps": STEPS, "solver_seed": SOLVER_SEED,
           "modes": {}}
    t = time.time()
    r = sb.run(isg.J, isg.h, isg.c0, "dsb", 32, STEPS, seed=SOLVER_SEED)
    E = energy.qubo_energy(q.a, q.b, sb.readout(r.x))
    out["modes"]["dsb"] = {"best": float(E.min()), "best_agent": int(np.argmin(E)),
                           "mean": float(E.mean()), "worst": float(E.max()),
                           "oracle_seconds": round(time.time() - t, 2)}
    print(out["modes"]["dsb"], flush=True)
    with open(os.path.join(HERE, "oracle_best_precision.json"), "w") as f:
        json.dump(out, f, indent=1)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "precision":
        precision()
        return
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
