"""Write the FP64 oracle's best QUBO energies used as time-to-target
references.  Calls only ``oracle`` and ``trackgen`` (the QUBOs are built by
the oracle's own builder; the SB runs by the C oracle ``oracle.sb_c``, which
is pinned bit for bit to ``oracle.sb``).

* oracle_best_plain.json: 200 particles, event seed 100; 256 agents,
  5000 steps, solver seed 0; bSB and dSB.
* oracle_best_precision.json: 1000 particles, event seed 200; dSB, all 1024
  agents, 5000 steps, solver seed 0.
* oracle_best_batching.json: the 512 batching events (particle counts
  20 + floor(981 U), U from seed 999; event seeds 1000-1511); dSB, 128
  agents, 3000 steps, solver seed 0, event e drawing its start with Philox
  counter word e (as the batched and one-event-at-a-time GPU solves do).

    python tests/golden/make_oracle_best.py [plain|precision|batching] [threads|workers]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import trackgen as tg  # noqa: E402
from oracle import energy, ising, qubo, sb, sb_c  # noqa: E402

SOLVER_SEED = 0


def _solve(q, mode, agents, steps, event=0, threads=0):
    isg = ising.from_qubo(q.a, q.b)
    t = time.time()
    x, _, used = sb_c.run(isg.J, isg.h, isg.c0, mode, agents, steps, seed=SOLVER_SEED,
                          event=event, threads=threads)
    E = energy.qubo_energy(q.a, q.b, sb.readout(x))
    return {"best": float(E.min()), "best_agent": int(np.argmin(E)), "mean": float(E.mean()),
            "worst": float(E.max()), "oracle_seconds": round(time.time() - t, 2),
            "threads": used}


def plain(threads):
    ev = tg.generate(tg.plain_spec(), 100)
    q = qubo.build_event(ev)
    out = {"event": "plain", "event_seed": 100, "n": q.n, "nnz": int(q.b.nnz),
           "agents": 256, "steps": 5000, "solver_seed": SOLVER_SEED, "modes": {}}
    for mode in ("bsb", "dsb"):
        out["modes"][mode] = _solve(q, mode, 256, 5000, threads=threads)
        print(mode, out["modes"][mode], flush=True)
    with open(os.path.join(HERE, "oracle_best_plain.json"), "w") as f:
        json.dump(out, f, indent=1)


def precision(threads):
    ev = tg.generate(tg.precision_spec(), 200)
    q = qubo.build_event(ev)
    out = {"event": "precision", "event_seed": 200, "n": q.n, "nnz": int(q.b.nnz),
           "agents": 1024, "agents_of_workload": 1024, "steps": 5000,
           "solver_seed": SOLVER_SEED, "modes": {"dsb": _solve(q, "dsb", 1024, 5000,
                                                               threads=threads)}}
    print(out["modes"]["dsb"], flush=True)
    with open(os.path.join(HERE, "oracle_best_precision.json"), "w") as f:
        json.dump(out, f, indent=1)


def _batching_event(arg):
    e, spec, seed = arg
    q = qubo.build_event(tg.generate(spec, seed))
    r = _solve(q, "dsb", 128, 3000, event=e, threads=1)
    return {"event": e, "event_seed": seed, "particles": spec.n_particles, "n": q.n,
            "nnz": int(q.b.nnz), "best": r["best"], "best_agent": r["best_agent"],
            "mean": r["mean"]}


def batching(workers):
    """Events in parallel processes (one host thread each): the oracle's
    builder is plain Python and dominates the time."""
    from multiprocessing import Pool
    M, K = 128, 3000
    jobs = [(e, spec, seed) for e, (spec, seed) in enumerate(tg.batching_specs())]
    jobs.sort(key=lambda j: -j[1].n_particles)     # largest first
    t0 = time.time()
    events = []
    with Pool(workers if workers > 0 else os.cpu_count()) as pool:
        for k, r in enumerate(pool.imap_unordered(_batching_event, jobs)):
            events.append(r)
            if k % 32 == 0:
                print(k, r, round(time.time() - t0, 1), flush=True)
    events.sort(key=lambda r: r["event"])
    out = {"workload": "batching", "events": len(events), "mode": "dsb", "agents": M,
           "steps": K, "solver_seed": SOLVER_SEED, "event_counter": "e (0..511)",
           "oracle_seconds": round(time.time() - t0, 1), "per_event": events}
    with open(os.path.join(HERE, "oracle_best_batching.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "plain"
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    {"plain": plain, "precision": precision, "batching": batching}[which](threads)
