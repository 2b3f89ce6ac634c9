"""Autotuner of the batched solver's schedule (sbt_batch_tuning).

For a batch of events (mode, coupling format, agents), every candidate
schedule -- which events run on the 512-thread step-kernel shape (two
workgroups per CU) rather than the 1024-thread one, how full a work item is
packed with agents, how many LDS words hold couplings past the register
capacity -- is planned and run on the GPU through the C ABI and timed with
HIP events on its stream.  A schedule changes no step arithmetic (only the
order of the FP64 energy sums), so every candidate must return the same
best energies to rounding (checked); the fastest is
written into the JSON tuning cache under the batch's key
(sbt_batch_tuning_key), where sbt_batch_tuning_lookup -- and through it
sbt_solve_batch, sbt_c0_scan and DeviceBatchSolver -- finds it.

    python -m paper_2402_14718_amd.autotune [--mode dsb] [--precision bf16]
        [--agents 128] [--steps 3000] [--reps 2] [--cache PATH]

tunes the batching workload (512 synthetic events of 20-1000 particles,
built by the GPU QUBO builder) and updates
paper_2402_14718_amd/tuning/batch_tuning.json.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(PKG, "tuning", "batch_tuning.json")
FORMAT = "sbtrack batch tuning 1"

SPLITS = (0, 1152, 2304, 4608)
FILLS = (1.0, 0.5)
TAILS = (8192, 4096)


def candidates():
    return [dict(split_n=s, fill=f, tail_words=t) for s, f, t in itertools.product(SPLITS, FILLS,
                                                                                   TAILS)]


def time_candidate(sbt, torch, qubos, mode, precision, params, cand, reps):
    """Seconds of one complete batched solve (prep, step kernels, selection)
    with this schedule, the best of `reps` after a warm-up, and the
    per-event best energies."""
    bs = sbt.DeviceBatchSolver(qubos, mode, precision, params, tuning=sbt.batch_tuning(**cand))
    bs.run()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.record()
        bs.run()
        e.record()
        torch.cuda.synchronize()
        best = min(best, b.elapsed_time(e) * 1e-3)
    energy = bs.result()["energy"]
    items = bs.n_items
    del bs
    return best, energy, items


def load_cache(path):
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
        if data.get("format") == FORMAT:
            return data
    return {"format": FORMAT, "entries": []}


def tune(qubos, mode="dsb", precision="bf16", agents=128, steps=3000, reps=2,
         cache_path=DEFAULT_CACHE, write=True, log=print):
    import torch

    import paper_2402_14718_amd as sbt

    params = sbt.solve_params(agents=agents, steps=steps, seed=0)
    key = sbt.batch_tuning_key([q.n for q in qubos], mode, precision, agents)
    trials, ref = [], None
    for cand in candidates():
        secs, energy, items = time_candidate(sbt, torch, qubos, mode, precision, params, cand,
                                             reps)
        if ref is None:
            ref = energy
        elif not np.allclose(energy, ref, rtol=1e-12, atol=1e-12):
            raise RuntimeError(f"schedule {cand} changed the results: a scheduling bug")
        trials.append(dict(cand, seconds=secs, work_items=items))
        log(f"[autotune] {cand} {secs * 1e3:.1f} ms ({items} items)")
    best = min(trials, key=lambda r: r["seconds"])
    default = next(r for r in trials
                   if r["split_n"] == 0 and r["fill"] == 1.0 and r["tail_words"] == 8192)
    entry = {"key": key, "split_n": best["split_n"], "tail_words": best["tail_words"],
             "fill": best["fill"], "seconds": best["seconds"],
             "default_seconds": default["seconds"], "steps": steps, "events": len(qubos),
             "tuned": time.strftime("%Y-%m-%d"), "trials": trials}
    if write:
        data = load_cache(cache_path)
        data["entries"] = [e for e in data["entries"] if e.get("key") != key] + [entry]
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, cache_path)
    return entry


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--mode", default="dsb", choices=["bsb", "dsb", "asb"])
    ap.add_argument("--precision", default="bf16", choices=["fp16", "bf16"])
    ap.add_argument("--agents", type=int, default=128)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    a = ap.parse_args(argv)
    import sys
    sys.path.insert(0, os.path.dirname(PKG))
    import torch
    # torch's device must be initialised before the library's first HIP call
    if not torch.cuda.is_available():
        raise SystemExit("autotune: no HIP device")
    import paper_2402_14718_amd as sbt
    import trackgen as tg
    qubos = [sbt.build_qubo_gpu(tg.generate(s, seed).hits_struct())[0]
             for s, seed in tg.batching_specs()]
    entry = tune(qubos, a.mode, a.precision, a.agents, a.steps, a.reps, a.cache)
    print(json.dumps({k: v for k, v in entry.items() if k != "trials"}))


if __name__ == "__main__":
    main()
