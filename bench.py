#!/usr/bin/env python3
"""Simulated-bifurcation throughput on one MI355X.

Workload ("plain"): one synthetic barrel event -- 10 layers at
r = 32 ... 1020 mm, 2 T, 200 helical particles (pT log-uniform 0.5-20 GeV,
|eta| < 1.5) plus 10% noise hits, event seed 100 -- turned into the triplet
QUBO by the library's host builder (not timed, as in the paper).  One bench
step is a complete solve of that QUBO in both SB forms, bSB and dSB, each
with 256 agents x 5000 symplectic-Euler steps: Ising preparation, Philox
start, all steps, FP64 energies of every agent and best-agent selection,
all on the GPU with the QUBO already resident in HBM.

Prints one JSON line with spin-updates/s (N * agents * steps * 2 forms per
bench step), the roofline position of the SB step kernel (timed live with
HIP events on its stream), the time to reach the FP64 oracle's best energy
within 0.5%, and the oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MI355X_FP32_VECTOR_TFLOPS = 157.3
# FP32 FMAs without the packed (two per lane) instructions, which the
# library's kernels are built without: 256 CUs x 4 SIMDs x 16 lanes x 2 flop
# x 2.4 GHz
MI355X_FP32_UNPACKED_TFLOPS = 78.6
MI355X_HBM_GBS = 8000.0
EVENT_SEED = 100
AGENTS = 256
SB_STEPS = 5000
SOLVER_SEED = 0
TTT_EVERY = 50


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def step_flops(n, nnz, agents, steps):
    """Useful FP32 flops of the SB steps: an FMA per stored coupling and
    8 per spin update (F + h, g x, c0 F - g x, y + dt f, x + dt a0 y)."""
    return float(steps) * agents * (2.0 * nnz + 8.0 * n)


def step_bytes(n, nnz, agents, steps):
    """Algorithmic bytes of the SB steps if state streamed through HBM:
    FP32 x, y read and written per spin update plus J (CSR FP32) per step."""
    return float(steps) * (16.0 * n * agents + 8.0 * nnz + 4.0 * (n + 1))


TTT_DEFINITIONS = {
    "checkpoint": "wall time of a complete solve (K steps, FP64 energies of every agent at every "
                  "50th step inside the timed solve) up to the first checkpoint whose best O(T) "
                  "is at or below E* + 0.005 |E*|, E* the FP64 oracle's best on the same event, "
                  "agents and seed; null if never reached",
    "ttt99": "the paper's time-to-target: target 99.9% of the lowest O(T) found (oracle and every "
             "GPU run of the form), agents as shots, P = 1 - (1 - p)^M per solve with p the "
             "fraction of agents at the target, TTT = t_solve ln(0.01) / ln(1 - P) (t_solve when "
             "P >= 0.99), minimised over K in a ladder of step counts",
}
TTT_LADDER = (25, 50, 100, 200, 500, 1000, 2000, 5000)


def load_golden(name):
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        return json.load(f)


def timed_runs(run, torch, reps=3):
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def ttt_checkpoint(s, K, target, torch, trace_of=lambda r: r["trace"]):
    """Checkpoint time-to-target of solver `s` (built with energy_every =
    TTT_EVERY and a trace): time of the solve scaled to the first checkpoint
    at or below `target`."""
    t = timed_runs(s.run, torch)
    tr = np.asarray(trace_of(s.result()))
    hit = np.nonzero(tr <= target)[0]
    if hit.size == 0:
        return {"steps": None, "seconds": None, "solve_seconds": t, "final": float(tr[-1])}
    steps = int(hit[0] + 1) * TTT_EVERY
    return {"steps": steps, "seconds": t * steps / K, "solve_seconds": t, "final": float(tr[-1])}


def ttt99(make, target, M, torch, energies_of=lambda s: s.result()["agent_energy"]):
    """The paper's TTT: agents as shots, 99% success probability."""
    best = None
    for K in TTT_LADDER:
        s = make(K)
        t = timed_runs(s.run, torch)
        p = float(np.mean(np.asarray(energies_of(s)) <= target))
        if p == 0.0:
            continue
        P = 1.0 - (1.0 - p) ** M
        tt = t if P >= 0.99 else t * np.log(0.01) / np.log1p(-P)
        if best is None or tt < best["seconds"]:
            best = {"steps": K, "seconds": float(tt), "p_agent": p, "solve_seconds": t}
    return best


def precision_form(sbt, tg, torch, np):
    """1000 particles (N ~ 8.5e3), dSB, 1024 agents x 5000 steps: plain FP32
    against the 16-bit-coupling forms (one-event batch), with the energy gap
    to the FP64 oracle (best of the first 32 agents) and both
    time-to-target definitions."""
    ref = load_golden("oracle_best_precision.json")
    ev = tg.generate(tg.precision_spec(), ref["event_seed"])
    q = sbt.build_qubo(ev.hits_struct())
    M, K = 1024, 5000
    e_star = ref["modes"]["dsb"]["best"]
    out = {"workload": "precision: 10-layer barrel, 1000 particles + 10% noise, event seed 200; "
                       "dSB, 1024 agents x 5000 steps", "n": q.n, "nnz": q.nnz,
           "oracle_best_32_agents": e_star}
    prm = lambda k, every=0: sbt.solve_params(agents=M, steps=k, seed=0, energy_every=every)
    forms = {
        "fp32": (lambda k, every=0: sbt.DeviceSolver(q, "dsb", prm(k, every),
                                                     want_trace=every > 0),
                 lambda r: r["energy"], lambda r: r["trace"], lambda r: r["agent_energy"]),
    }
    for prec in ("fp16", "bf16"):
        forms[prec] = (lambda k, every=0, prec=prec: sbt.DeviceBatchSolver(
                           [q], "dsb", prec, prm(k, every), want_agent_energy=True,
                           want_trace=every > 0),
                       lambda r: float(r["energy"][0]), lambda r: r["trace"][0],
                       lambda r: r["agent_energy"][0])
    for name, (make, best_of, trace_of, agents_of) in forms.items():
        s = make(K)
        t = timed_runs(s.run, torch, reps=2)
        e = best_of(s.result())
        out[name] = {"kernel": getattr(s, "kernel", "sb_batch"), "seconds": t,
                     "spin_updates_per_s": q.n * M * K / t, "best": e, "gap_to_oracle": e - e_star,
                     "ttt_checkpoint": ttt_checkpoint(make(K, TTT_EVERY), K,
                                                      e_star + 0.005 * abs(e_star), torch,
                                                      trace_of)}
        if name == "fp32" and out[name]["kernel"] == "stream":
            # one streaming launch per step: its duration from the library's
            # step events, against the step's algorithmic HBM bytes
            b, ev_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            b.record()
            ev_.record()
            torch.cuda.synchronize()
            s._dr.step_begin, s._dr.step_end = b.cuda_event, ev_.cuda_event
            s.run()
            torch.cuda.synchronize()
            s._dr.step_begin = s._dr.step_end = None
            launch_s = b.elapsed_time(ev_) * 1e-3 / K
            byts = stream_bytes_dsb(q.n, q.nnz, M)
            achieved = byts / launch_s / 1e9
            out[name]["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": MI355X_HBM_GBS,
                                     "unit": "GB/s", "frac": achieved / MI355X_HBM_GBS,
                                     "traffic": measured_traffic("sb_stream_precision_dsb.md"),
                                     "kernel": "sb_stream",
                                     "launch_ms": launch_s * 1e3, "bytes_per_launch": byts}
        del s
    e_low = min([e_star] + [out[n]["best"] for n in forms])
    out["ttt99_target"] = 0.999 * e_low
    for name, (make, best_of, trace_of, agents_of) in forms.items():
        out[name]["ttt99"] = ttt99(make, 0.999 * e_low, M, torch,
                                   lambda s, f=agents_of: f(s.result()))
    return out


def batched_form(sbt, tg, torch, np, with_fp32=True, gpu_build=True):
    """512 events of 20-1000 particles, dSB, 128 agents x 3000 steps: one
    persistent batched kernel (FP16 / BF16 couplings) against plain FP32
    solving the events one at a time.  Per-event energies are compared with
    the plain FP32 results (the FP64 oracle cannot run this batch); the
    checkpoint time-to-target is the time until every event's best-so-far
    FP64 O(T) is within 0.5% of its FP32 best (FP32: the sum over events of
    each solve's time to its own first such checkpoint)."""
    specs = tg.batching_specs()
    hits = [tg.generate(s, seed).hits_struct() for s, seed in specs]
    # QUBO construction of every event on the GPU (wall time, downloads
    # included); the host builder timed on a sample of events, whose
    # structure must match (on every event, and no GPU construction, with
    # --batch-host-build)
    sample = 64 if gpu_build else len(hits)
    t0 = time.perf_counter()
    host = [sbt.build_qubo(h) for h in hits[:sample]]
    host_sample_s = time.perf_counter() - t0
    if gpu_build:
        t0 = time.perf_counter()
        built = [sbt.build_qubo_gpu(h) for h in hits]
        gpu_build_s = time.perf_counter() - t0
    else:  # host-built QUBOs (profiling runs: only the solver's kernels on the GPU)
        built, gpu_build_s = [(q, 0.0) for q in host], None
    qs = [q for q, _ in built]
    same = all(np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col) and
               np.array_equal(a.trip_hits, b.trip_hits) for a, b in zip(qs, host))
    M, K = 128, 3000
    sum_n = sum(q.n for q in qs)
    sum_nnz = sum(q.nnz for q in qs)
    out = {"workload": "batching: 512 events, 20 + floor(981 U) particles (U from seed 999), "
                       "event seeds 1000-1511; dSB, 128 agents x 3000 steps",
           "events": len(qs), "sum_n": sum_n, "max_n": max(q.n for q in qs),
           "qubo_build": {"gpu_all_events_s": gpu_build_s,
                          "gpu_device_s": float(sum(d for _, d in built)) if gpu_build else None,
                          "host_all_events_s_from_sample": host_sample_s * len(qs) / sample,
                          "host_sample": f"first {sample} events, {host_sample_s:.2f} s",
                          "same_structure_on_sample": bool(same) if gpu_build else None}}
    if with_fp32:
        plain = [sbt.DeviceSolver(q, "dsb", sbt.solve_params(agents=M, steps=K, seed=0, event=e))
                 for e, q in enumerate(qs)]

        def run_plain():
            for s in plain:
                s.run()

        t = timed_runs(run_plain, torch, reps=1)
        e32 = np.array([float(s.best_energy.item()) for s in plain])
        out["fp32_one_event_at_a_time"] = {"seconds": t, "spin_updates_per_s": sum_n * M * K / t}
        del plain
        # checkpoint time-to-target against each event's FP32 best: every
        # event's best-so-far within 0.5% of it
        target = e32 + 0.005 * np.abs(e32)
        traced = [sbt.DeviceSolver(q, "dsb", sbt.solve_params(agents=M, steps=K, seed=0, event=e,
                                                             energy_every=TTT_EVERY),
                                   want_trace=True) for e, q in enumerate(qs)]
        for s in traced:
            s.run()
        torch.cuda.synchronize()
        pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in traced]
        for s, (b, e) in zip(traced, pairs):
            b.record()
            s.run()
            e.record()
        torch.cuda.synchronize()
        ttt32 = 0.0
        for e, (s, (b0, e0)) in enumerate(zip(traced, pairs)):
            hit = np.nonzero(s.result()["trace"] <= target[e])[0]
            ttt32 += b0.elapsed_time(e0) * 1e-3 * (hit[0] + 1) * TTT_EVERY / K
        out["fp32_one_event_at_a_time"]["ttt_checkpoint_all_events"] = ttt32
        del traced
        log("batched form: FP32 one event at a time done")
    for prec in ("fp16", "bf16"):
        bs = sbt.DeviceBatchSolver(qs, "dsb", prec, sbt.solve_params(agents=M, steps=K, seed=0))
        tb = timed_runs(bs.run, torch, reps=2)
        # the batch kernel's own duration, on its stream, from the library's step events
        b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.record()
        e.record()
        torch.cuda.synchronize()
        bs._dr.step_begin, bs._dr.step_end = b.cuda_event, e.cuda_event
        bs.run()
        torch.cuda.synchronize()
        bs._dr.step_begin = bs._dr.step_end = None
        launch_s = b.elapsed_time(e) * 1e-3
        flops = float(K) * M * (2.0 * sum_nnz + 8.0 * sum_n)
        achieved = flops / launch_s / 1e12
        out[prec] = {"seconds": tb, "spin_updates_per_s": sum_n * M * K / tb,
                     "work_items": bs.n_items,
                     "roofline": {"bound": "alu", "achieved": achieved,
                                  "peak": MI355X_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                                  "frac": achieved / MI355X_FP32_VECTOR_TFLOPS,
                                  "peak_without_packed_fp32": MI355X_FP32_UNPACKED_TFLOPS,
                                  "frac_without_packed_fp32": achieved / MI355X_FP32_UNPACKED_TFLOPS,
                                  "traffic": measured_traffic(f"sb_batch_batching_{prec}.md"),
                                  "lds": measured_lds(f"sb_batch_batching_{prec}.md"),
                                  "kernel": "sb_batch", "launch_ms": launch_s * 1e3}}
        if with_fp32:
            bt = sbt.DeviceBatchSolver(qs, "dsb", prec, sbt.solve_params(
                agents=M, steps=K, seed=0, energy_every=TTT_EVERY), want_trace=True)
            tt = timed_runs(bt.run, torch, reps=1)
            tr = bt.result()["trace"]
            ok = np.all(tr <= target[:, None], axis=0)
            out[prec]["ttt_checkpoint_all_events"] = (
                None if not ok.any() else tt * (int(np.argmax(ok)) + 1) * TTT_EVERY / K)
            del bt
            gap = (bs.result()["energy"] - e32) / np.abs(e32)
            out[prec].update({"speedup_vs_fp32": t / tb,
                              "rel_energy_gap_vs_fp32": {"mean": float(gap.mean()),
                                                         "max": float(gap.max()),
                                                         "min": float(gap.min())},
                              "events_within_0.5pct_of_fp32": int(np.sum(gap <= 0.005))})
        log(f"batched form: {prec} batch done")
    # hits to every event's best spins on the GPU: construction + one batch
    out["end_to_end_fp16_s"] = None if gpu_build_s is None else gpu_build_s + out["fp16"]["seconds"]
    return out


def stream_bytes(n, nnz, agents, jbytes):
    """Algorithmic HBM bytes of one streaming-kernel launch (one SB step):
    x, y read and written per spin update, each coupling's column and value
    once, h, row pointers and the per-row scale once."""
    return 16.0 * n * agents + (4.0 + jbytes) * nnz + 12.0 * n


def stream_bytes_dsb(n, nnz, agents):
    """Algorithmic HBM bytes of one dSB streaming launch: x, y read and
    written in place per spin update, the 64-agent sign words of every spin
    read once and written once, each coupling's column and value once, h,
    row pointers and the per-row scale once."""
    words = (agents + 63) // 64
    return 16.0 * n * agents + 16.0 * n * words + 8.0 * nnz + 12.0 * n


def stress_form(sbt, tg, torch, np, K=10000):
    """5000 particles (N ~ 2.1e5), bSB, 512 agents x 10000 steps on the
    streaming kernel: FP8 couplings (the workload's storage) and FP32, spins
    in azimuth order, FP64 energies of every agent on the GPU."""
    ev = tg.generate(tg.stress_spec(), 300)
    hits = ev.hits_struct()
    bp = sbt.build_params_default()
    bp.z0_max = tg.STRESS_Z0_MAX
    t0 = time.perf_counter()
    q0 = sbt.build_qubo(hits, bp)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    qg, t_gpu_dev = sbt.build_qubo_gpu(hits, bp)
    t_gpu = time.perf_counter() - t0
    same = bool(qg.n == q0.n and np.array_equal(qg.col, q0.col) and
                np.array_equal(qg.row_ptr, q0.row_ptr))
    del qg
    t0 = time.perf_counter()
    q = sbt.permute_qubo(q0, sbt.phi_order(q0, hits))
    t_order = time.perf_counter() - t0
    del q0
    M = 512
    out = {"workload": "stress: 10-layer barrel, 5000 particles + 20% noise, |eta| < 2, event "
                       f"seed 300, doublet |z0| <= 300 mm; bSB, 512 agents x {K} steps, "
                       "spins in azimuth order",
           "n": q.n, "nnz": q.nnz, "host_build_s": t_build, "host_order_s": t_order,
           "gpu_build_s": t_gpu, "gpu_build_device_s": t_gpu_dev,
           "gpu_build_same_structure": same}
    for prec in ("fp8", "fp32"):
        s = sbt.DeviceSolver(q, "bsb", sbt.solve_params(agents=M, steps=K, seed=0,
                                                         kernel="stream", precision=prec))
        b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.record()
        e.record()
        torch.cuda.synchronize()
        s._dr.step_begin, s._dr.step_end = b.cuda_event, e.cuda_event
        t0 = time.perf_counter()
        s.run()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s._dr.step_begin = s._dr.step_end = None
        launch_s = b.elapsed_time(e) * 1e-3 / K
        r = s.result()
        E = np.sort(r["agent_energy"])
        byts = stream_bytes(q.n, q.nnz, M, 1 if prec == "fp8" else 4)
        achieved = byts / launch_s / 1e9
        out[prec] = {"seconds": wall, "spin_updates_per_s": q.n * M * K / wall,
                     "best": r["energy"], "mean_best_32": float(E[:32].mean()),
                     "roofline": {"bound": "hbm", "achieved": achieved, "peak": MI355X_HBM_GBS,
                                  "unit": "GB/s", "frac": achieved / MI355X_HBM_GBS,
                                  "traffic": measured_traffic(f"sb_stream_stress_{prec}.md"),
                                  "kernel": "sb_stream_v4", "launch_ms": launch_s * 1e3,
                                  "bytes_per_launch": byts}}
        del s
        torch.cuda.empty_cache()
    out["fp8_rel_gap_vs_fp32"] = (out["fp8"]["best"] - out["fp32"]["best"]) / abs(out["fp32"]["best"])
    return out


def c0_scan_form(sbt, q, torch):
    """Automatic c0 scan on the plain event (Results: fixed c0 or a scan):
    c0 * 2^k for k = -3..3, dSB and bSB, FP16 batch, 256 agents x 5000
    steps, every copy from the same start."""
    ref = load_golden("oracle_best_plain.json")
    factors = [2.0 ** k for k in range(-3, 4)]
    out = {"factors": factors}
    for mode in ("dsb", "bsb"):
        t0 = time.perf_counter()
        s = sbt.c0_scan(q, mode, factors, "fp16", agents=AGENTS, steps=SB_STEPS, seed=SOLVER_SEED)
        out[mode] = {"energy": s["energy"].tolist(), "best_factor": s["factor"],
                     "seconds": time.perf_counter() - t0,
                     "oracle_best_fixed_c0": ref["modes"][mode]["best"]}
    return out


def measured_traffic(profile_name):
    """HBM bytes per launch from the committed rocprofv3 counter record, or
    None when the kernel's sources changed after the counters were taken."""
    from paper_2402_14718_amd import rocprof_summary as rs
    rec = rs.read_record(os.path.join(ROOT, "profiles", profile_name))
    if not rec or rec.get("sources_sha") != rs.sources_hash(rec["family"]):
        return None
    return rec["hbm_bytes_per_launch"]


def measured_lds(profile_name):
    """LDS use of the kernel from the committed rocprofv3 counter record, as
    fractions of the chip's CU cycles (GRBM_GUI_ACTIVE comes summed over the
    8 XCDs): cycles the LDS serves indexed accesses, and of those the cycles
    stalled on bank conflicts.  None when the record lacks those counters or
    the kernel's sources changed after they were taken."""
    from paper_2402_14718_amd import rocprof_summary as rs
    rec = rs.read_record(os.path.join(ROOT, "profiles", profile_name))
    if not rec or rec.get("sources_sha") != rs.sources_hash(rec["family"]):
        return None
    sq = rec.get("sq") or {}
    if "SQ_LDS_IDX_ACTIVE" not in sq or "GRBM_GUI_ACTIVE" not in sq:
        return None
    cu_cycles = sq["GRBM_GUI_ACTIVE"] / 8 * 256
    return {"busy_frac": sq["SQ_LDS_IDX_ACTIVE"] / cu_cycles,
            "bank_conflict_frac": sq.get("SQ_LDS_BANK_CONFLICT", 0.0) / cu_cycles,
            "source": f"profiles/{profile_name}"}


def _sized_run(run_one, target_s):
    """Grow a bSB run until it takes a second, then time bSB + dSB at the
    step count that fills about target_s; returns (steps, seconds)."""
    k = 25
    while True:
        t0 = time.perf_counter()
        run_one("bsb", k)
        dt = time.perf_counter() - t0
        if dt >= 1.0:
            break
        k *= 4
    k = max(20, int(k * target_s / (2.0 * dt)))
    t0 = time.perf_counter()
    for mode in ("bsb", "dsb"):
        run_one(mode, k)
    return k, time.perf_counter() - t0


def _oracle_form_rate(qs, mode, agents, target_s, threads_used):
    """C oracle (all host threads) on the QUBOs `qs`: spin-updates/s from the
    difference of a 2-step run and a longer one (x4 until the difference
    reaches half of target_s), so the per-run copies of the state and the
    per-call overheads cancel."""
    import scipy.sparse as sp

    from oracle import ising as oising
    from oracle import sb_c

    isgs = [oising.from_qubo(q.a, sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n)))
            for q in qs]

    def run(k):
        t0 = time.perf_counter()
        for e, isg in enumerate(isgs):
            threads_used[0] = sb_c.run(isg.J, isg.h, isg.c0, mode, agents, k, seed=SOLVER_SEED,
                                       event=e)[2]
        return time.perf_counter() - t0

    t_lo = run(2)
    k = 8
    dt = run(k) - t_lo
    while dt < target_s / 2 and k < 1 << 20:
        k *= 4
        dt = run(k) - t_lo
    return {"spin_updates_per_s": sum(q.n for q in qs) * agents * (k - 2) / dt, "mode": mode,
            "agents": agents, "steps": f"{k} minus 2", "seconds": dt}


def cpu_forms_baseline(sbt, tg, target_s=4.0):
    """The C oracle on every host thread for the precision, batching and
    stress workloads (a bounded number of steps each; per-step cost is
    constant, so the rate carries over to the full step counts)."""
    used = [0]
    ref = load_golden("oracle_best_precision.json")
    out = {"precision": _oracle_form_rate(
        [sbt.build_qubo(tg.generate(tg.precision_spec(), ref["event_seed"]).hits_struct())],
        "dsb", 1024, target_s, used)}
    qs = [sbt.build_qubo_gpu(tg.generate(sp_, seed).hits_struct())[0]
          for sp_, seed in tg.batching_specs()]
    out["batching"] = _oracle_form_rate(qs, "dsb", 128, target_s, used)
    del qs
    ev = tg.generate(tg.stress_spec(), 300)
    bp = sbt.build_params_default()
    bp.z0_max = tg.STRESS_Z0_MAX
    q = sbt.build_qubo_gpu(ev.hits_struct(), bp)[0]
    q = sbt.permute_qubo(q, sbt.phi_order(q, ev.hits_struct()))
    out["stress"] = _oracle_form_rate([q], "bsb", 512, target_s, used)
    out["threads"] = used[0]
    return out


def cpu_baseline(q, target_s=8.0):
    """The FP64 oracle on the host, both forms, all 256 agents, for a bounded
    number of steps, as spin-updates/s: the C oracle with the agents spread
    over every host thread OpenMP is given (the reported value), and the
    NumPy/SciPy oracle on one thread (reported beside it)."""
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import ising as oising
    from oracle import sb as osb
    from oracle import sb_c

    if not os.path.exists(sb_c.LIB):
        sb_c.build()
    b = sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n))
    isg = oising.from_qubo(q.a, b)
    used = [0]

    def run_c(mode, k):
        used[0] = sb_c.run(isg.J, isg.h, isg.c0, mode, AGENTS, k, seed=SOLVER_SEED)[2]

    k2, dt2 = _sized_run(run_c, target_s)
    with threadpool_limits(limits=1):
        k1, dt1 = _sized_run(lambda mode, k: osb.run(isg.J, isg.h, isg.c0, mode, AGENTS, k,
                                                     seed=SOLVER_SEED), target_s)
    ups2 = 2.0 * q.n * AGENTS * k2 / dt2
    ups1 = 2.0 * q.n * AGENTS * k1 / dt1
    return {"value": ups2, "unit": "spin-updates/s", "cores": used[0], "kind": "oracle",
            "sample": f"C FP64 oracle (oracle/sb_omp.c, OpenMP over agents), bSB+dSB, {AGENTS} "
                      f"agents x {k2} steps on the same event ({dt2:.1f} s, {used[0]} threads)",
            "python_oracle_one_thread": {
                "value": ups1, "unit": "spin-updates/s", "cores": 1,
                "sample": f"NumPy/SciPy FP64 oracle, bSB+dSB, {AGENTS} agents x {k1} steps "
                          f"({dt1:.1f} s)"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed bench steps")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttt", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision (1000 particles), batched (512 events) and stress "
                         "(5000 particles) forms")
    ap.add_argument("--only", choices=["precision", "batched", "stress"],
                    help="run only this form and print it (for profiling one kernel)")
    ap.add_argument("--batch-skip-fp32", action="store_true",
                    help="batched form without the FP32 one-event-at-a-time comparison "
                         "(for counter collection)")
    ap.add_argument("--batch-host-build", action="store_true",
                    help="batched form on host-built QUBOs, without the GPU builder's "
                         "launches (for counter collection)")
    ap.add_argument("--stress-steps", type=int, default=10000,
                    help="SB steps of the stress form (10000 is the workload's)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "resident", "stream"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB buffer 3 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; the solver shards over agents with no per-step "
              "communication, so --gpus N > 1 is not run", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2402_14718_amd as sbt
    import trackgen as tg

    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.only:
        form = {"precision": lambda: precision_form(sbt, tg, torch, np),
                "batched": lambda: batched_form(sbt, tg, torch, np, not args.batch_skip_fp32,
                                                not args.batch_host_build),
                "stress": lambda: stress_form(sbt, tg, torch, np, args.stress_steps)}[args.only]
        print(json.dumps({f"{args.only}_form": form()}), flush=True)
        return
    log("building the event QUBO on the host")
    ev = tg.generate(tg.plain_spec(), EVENT_SEED)
    q = sbt.build_qubo(ev.hits_struct())
    log(f"N={q.n} nnz={q.nnz} agents={AGENTS} sb_steps={SB_STEPS}")

    solvers = []
    for mode in ("bsb", "dsb"):
        p = sbt.solve_params(agents=AGENTS, steps=SB_STEPS, seed=SOLVER_SEED, kernel=args.kernel)
        solvers.append(sbt.DeviceSolver(q, mode, p))
    kernel = solvers[0].kernel
    stream = torch.cuda.current_stream()

    def event_pair():
        b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.record(stream)   # materialise the HIP events so their handles exist
        e.record(stream)
        return b, e

    for _ in range(args.warmup):
        for s in solvers:
            s.run()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps), kernel={kernel}")

    pairs = [[event_pair() for _ in solvers] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for s, (b, e) in zip(solvers, pairs[k]):
            s._dr.step_begin = b.cuda_event
            s._dr.step_end = e.cuda_event
            s.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = [b.elapsed_time(e) for row in pairs for (b, e) in row]
    for s in solvers:
        s._dr.step_begin = s._dr.step_end = None
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

    updates = 2.0 * q.n * AGENTS * SB_STEPS * args.steps
    value = updates / elapsed
    launches_per_solve = 1 if kernel == "resident" else SB_STEPS
    phase_s = float(np.mean(step_ms)) * 1e-3
    launch_s = phase_s / launches_per_solve
    flops = step_flops(q.n, q.nnz, AGENTS, SB_STEPS) / launches_per_solve
    bytes_ = step_bytes(q.n, q.nnz, AGENTS, SB_STEPS) / launches_per_solve
    if kernel == "resident":
        achieved = flops / launch_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": MI355X_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / MI355X_FP32_VECTOR_TFLOPS,
                "peak_without_packed_fp32": MI355X_FP32_UNPACKED_TFLOPS,
                "frac_without_packed_fp32": achieved / MI355X_FP32_UNPACKED_TFLOPS,
                "traffic": measured_traffic("sb_resident_reg_plain.md"),
                "lds": measured_lds("sb_resident_reg_plain.md"),
                "kernel": "sb_resident_reg", "launch_ms": launch_s * 1e3,
                "state_bytes_if_streamed_GBs": bytes_ / launch_s / 1e9}
    else:
        achieved = bytes_ / launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": MI355X_HBM_GBS, "unit": "GB/s",
                "frac": achieved / MI355X_HBM_GBS, "traffic": None, "kernel": "sb_stream",
                "launch_ms": launch_s * 1e3}

    result = {
        "metric": "SB spin-updates/s + time-to-best-energy, BF16/FP8 batched vs plain FP32 SB",
        "value": value, "unit": "spin-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain: 10-layer barrel, 200 particles + 10% noise, event seed 100; "
                               "bSB and dSB, 256 agents x 5000 steps, CSR FP32",
                   "n": q.n, "nnz": q.nnz, "agents": AGENTS, "sb_steps": SB_STEPS,
                   "forms": ["bsb", "dsb"], "kernel": kernel},
        "roofline": roof,
    }

    if not args.no_ttt:
        ref = load_golden("oracle_best_plain.json")
        ttt = {"definitions": TTT_DEFINITIONS}
        for mode in ("bsb", "dsb"):
            e_star = ref["modes"][mode]["best"]
            mk = lambda K, every=0, mode=mode: sbt.DeviceSolver(
                q, mode, sbt.solve_params(agents=AGENTS, steps=K, seed=SOLVER_SEED,
                                          kernel=args.kernel, energy_every=every),
                want_trace=every > 0)
            ck = ttt_checkpoint(mk(SB_STEPS, TTT_EVERY), SB_STEPS, e_star + 0.005 * abs(e_star),
                                torch)
            e_low = min(e_star, ck["final"])
            ttt[mode] = {"oracle_best": e_star, "checkpoint": ck, "ttt99_target": 0.999 * e_low,
                         "ttt99": ttt99(mk, 0.999 * e_low, AGENTS, torch)}
        # CPU comparator (the paper's SA baseline role): TTT99 over sweeps
        e_low = min(ref["modes"][m]["best"] for m in ("bsb", "dsb"))
        target = 0.999 * e_low
        best = None
        for sweeps in (10, 30, 100, 300, 1000):
            r = sbt.anneal_cpu(q, shots=50, sweeps=sweeps, seed=SOLVER_SEED)
            p_s = float(np.mean(r["shot_energy"] <= target))
            if p_s == 0.0:
                continue
            P = 1.0 - (1.0 - p_s) ** 50
            tt = r["elapsed_s"] if P >= 0.99 else r["elapsed_s"] * np.log(0.01) / np.log1p(-P)
            if best is None or tt < best["seconds"]:
                best = {"sweeps": sweeps, "seconds": float(tt), "p_shot": p_s,
                        "run_seconds": r["elapsed_s"]}
        ttt["sa_cpu"] = {"target": target, "shots": 50, "cores": os.cpu_count(),
                         "ttt99": best,
                         "note": "single-flip Metropolis annealing on the host, all cores"}
        result["time_to_target"] = ttt
        log("time-to-target done")

    if not args.no_forms:
        result["precision_form"] = precision_form(sbt, tg, torch, np)
        log("precision form done")
        result["batched_form"] = batched_form(sbt, tg, torch, np)
        log("batched form done")
        result["stress_form"] = stress_form(sbt, tg, torch, np, args.stress_steps)
        log("stress form done")
        result["c0_scan"] = c0_scan_form(sbt, q, torch)
        log("c0 scan done")

    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)")
        result["cpu_baseline"] = cpu_baseline(q)
        if not args.no_forms:
            log("timing the C oracle on the other workloads (bounded samples)")
            result["cpu_baseline"]["forms"] = cpu_forms_baseline(sbt, tg)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
