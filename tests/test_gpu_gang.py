"""GPU parity of events solved as gangs of row bands (events too large for
one workgroup's 9216 slots, or any event with a small band_rows tuning):
the bands of one (event, agent) run at once on different workgroups and
exchange positions through HBM with one barrier per step.

* The same arithmetic per (spin, agent) as the one-workgroup path, so a
  gang must reproduce that path's positions bit for bit (small events
  forced into gangs by band_rows), and its energies to rounding.
* Against the FP64 oracle with the same rounded couplings: trajectories
  within 1e-5 over 50 steps (close calls exempt, >= 90% of agents), exact
  FP64 energies of the returned spins (1e-9), checkpoint energies at 1e-9,
  on a batch holding an 11361-variable event beside small ones.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import trackgen as tg
from oracle import energy as oenergy
from oracle import ising as oising
from oracle import quant as oquant
from oracle import sb as osb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2402_14718_amd as sbt  # noqa: E402

ROUND = {"fp16": oquant.fp16_couplings, "bf16": oquant.bf16_couplings}


def _q(spec, seed):
    return sbt.build_qubo(tg.generate(spec, seed).hits_struct())


@pytest.fixture(scope="module")
def big_batch():
    qs = [_q(tg.plain_spec(60), 2), _q(tg.plain_spec(1200), 77), _q(tg.plain_spec(300), 8)]
    assert qs[1].n > 9216
    return qs


def _solve(qs, mode, prec, M, K, seed, tuning, dt=1.0, every=0):
    ds = sbt.DeviceBatchSolver(qs, mode, prec, sbt.solve_params(agents=M, steps=K, seed=seed,
                                                               dt=dt, energy_every=every),
                               want_agent_energy=True, want_agent_state=True,
                               want_trace=every > 0, tuning=tuning)
    ds.run()
    return ds.result(), ds


@pytest.mark.parametrize("mode,prec", [("dsb", "bf16"), ("bsb", "fp16"), ("asb", "bf16")])
def test_forced_gangs_equal_the_one_workgroup_path(mode, prec):
    """band_rows = 300 cuts the 1480-variable plain event into 5 bands and
    the 600-variable one into 2; 64 agents give 64 gangs each (more items
    than CUs, so gangs queue behind gangs)."""
    qs = [_q(tg.plain_spec(), 100), _q(tg.plain_spec(80), 3), _q(tg.tiny_spec(), 4)]
    dt = 0.1 if mode == "asb" else 1.0
    M, K = 64, 150
    ref, _ = _solve(qs, mode, prec, M, K, 5, sbt.batch_tuning(), dt=dt, every=25)
    got, ds = _solve(qs, mode, prec, M, K, 5, sbt.batch_tuning(band_rows=300), dt=dt, every=25)
    assert ds.n_items > 256
    for e in range(len(qs)):
        assert np.array_equal(got["agent_x"][e], ref["agent_x"][e]), e
        assert np.array_equal(got["agent_T"][e], ref["agent_T"][e]), e
    for k in ("energy", "agent_energy", "trace", "agent_trace"):
        assert np.allclose(got[k], ref[k], rtol=1e-12, atol=1e-12), k
    assert np.array_equal(got["best_agent"], ref["best_agent"])


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("mode", ["bsb", "dsb"])
@pytest.mark.parametrize("dt", [1.0, 0.1])
def test_large_event_trajectories_match_oracle(big_batch, prec, mode, dt):
    M, K, seed = 32, 50, 23
    r, _ = _solve(big_batch, mode, prec, M, K, seed, None, dt=dt)
    for e, q in enumerate(big_batch):
        b = sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n))
        isg = oising.from_qubo(q.a, b)
        ref = osb.run(ROUND[prec](isg.J), isg.h, isg.c0, mode, M, K, dt=dt, seed=seed, event=e,
                      margin_steps=K)
        x = r["agent_x"][e]
        err = np.linalg.norm(x - ref.x, axis=0) / np.linalg.norm(ref.x, axis=0)
        close = ref.wall_margin < 1e-6
        if mode == "dsb":
            close |= ref.sign_margin < 1e-6
        assert np.all((err <= 1e-5) | close), (e, err.max())
        assert np.mean(err <= 1e-5) >= 0.9
        T = r["agent_T"][e]
        assert np.array_equal(T, (x >= 0).astype(np.int8))
        e_or = oenergy.qubo_energy(q.a, b, T)
        assert np.allclose(r["agent_energy"][e], e_or, rtol=1e-12, atol=1e-9)
        assert r["best_agent"][e] == oenergy.best_agent(e_or)
        assert np.array_equal(r["T"][e], T[:, r["best_agent"][e]])


def test_large_event_checkpoints_match_oracle(big_batch):
    M, K, every, seed = 16, 30, 7, 4
    r, _ = _solve(big_batch, "dsb", "bf16", M, K, seed, None, dt=0.1, every=every)
    for e, q in enumerate(big_batch):
        b = sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n))
        isg = oising.from_qubo(q.a, b)
        ref = osb.run(ROUND["bf16"](isg.J), isg.h, isg.c0, "dsb", M, K, dt=0.1, seed=seed,
                      event=e, margin_steps=K, ckpt_every=every, qubo=(q.a, b))
        clear = ((ref.wall_margin >= 1e-6) & (ref.readout_margin >= 1e-6) &
                 (ref.sign_margin >= 1e-6))
        tol = 1e-9 * np.maximum(1.0, np.abs(ref.agent_trace))
        match = np.all(np.abs(r["agent_trace"][e] - ref.agent_trace) <= tol, axis=0)
        assert np.all(match | ~clear), e
        assert np.mean(match) >= 0.9
        assert np.array_equal(r["trace"][e],
                              np.minimum.accumulate(r["agent_trace"][e].min(axis=1)))


def test_large_event_full_length_quality(big_batch):
    """128 agents x 3000 steps on the large event: best within 0.5% of the
    plain FP32 solve of the same event, same agents and seed."""
    M, K = 128, 3000
    r, _ = _solve(big_batch[1:2], "dsb", "bf16", M, K, 0, None)
    f = sbt.DeviceSolver(big_batch[1], "dsb", sbt.solve_params(agents=M, steps=K, seed=0))
    f.run()
    e32 = f.result()["energy"]
    assert r["energy"][0] <= e32 + 0.005 * abs(e32)
    assert np.all(np.isfinite(r["agent_energy"]))


def test_host_batch_with_a_large_event(big_batch):
    h = sbt.solve_batch(big_batch, "dsb", "fp16", agents=8, steps=40, seed=2)
    d, _ = _solve(big_batch, "dsb", "fp16", 8, 40, 2, None)
    assert np.allclose(h["energy"], d["energy"], rtol=1e-12)


def test_target_mode_stops_each_event_at_its_target():
    """Target mode, with a target that every event reaches at its first
    checkpoint: every agent's checkpoint energies are a prefix of the free
    solve's (the rest NaN: its work stopped), its returned energy is that of
    the last checkpoint it reached, and the best-so-far trace reaches the
    target at the first checkpoint.  With an unreachable target the solve
    equals the free one.  Both paths: events on one workgroup (the items of
    an event stop through the event's flag, so where an item stops depends
    on timing) and events forced into gangs (each agent's gang on its own
    energy)."""
    qs = [_q(tg.plain_spec(), 100), _q(tg.plain_spec(80), 3), _q(tg.tiny_spec(), 4)]
    M, K, every = 32, 200, 20
    for tuning in (sbt.batch_tuning(), sbt.batch_tuning(band_rows=500)):
        free, _ = _solve(qs, "dsb", "bf16", M, K, 3, tuning, every=every)
        first = free["agent_trace"][:, 0, :].min(axis=1)
        ds = sbt.DeviceBatchSolver(qs, "dsb", "bf16", sbt.solve_params(
            agents=M, steps=K, seed=3, energy_every=every), want_agent_energy=True,
            want_agent_state=True, want_trace=True, tuning=tuning, target=first + 1e-9)
        ds.run()
        r = ds.result()
        stopped = 0
        for e in range(len(qs)):
            at, ft = r["agent_trace"][e], free["agent_trace"][e]
            assert r["trace"][e][0] <= first[e] + 1e-9
            for m in range(M):
                reached = ~np.isnan(at[:, m])
                n_ok = int(reached.sum())
                assert n_ok >= 1 and np.all(reached[:n_ok]), (e, m)   # a prefix
                assert np.allclose(at[:n_ok, m], ft[:n_ok, m], rtol=1e-12), (e, m)
                assert np.isclose(r["agent_energy"][e][m], at[n_ok - 1, m], rtol=1e-12)
                stopped += n_ok < K // every
        assert stopped > 0
        never = sbt.DeviceBatchSolver(qs, "dsb", "bf16", sbt.solve_params(
            agents=M, steps=K, seed=3, energy_every=every), want_agent_energy=True,
            want_agent_state=True, want_trace=True, tuning=tuning, target=np.full(3, -1e30))
        never.run()
        rn = never.result()
        for e in range(len(qs)):
            assert np.array_equal(rn["agent_x"][e], free["agent_x"][e])
        assert np.allclose(rn["energy"], free["energy"], rtol=1e-12)
