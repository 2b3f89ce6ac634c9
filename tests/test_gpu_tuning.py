"""GPU checks of the batch tuning (sbt_batch_tuning) through the C ABI.

A schedule moves events between work items and step-kernel shapes but
changes no agent's step arithmetic, so every tuning must give bit-identical
positions and assignments; the FP64 energies are summed over the spins a
workgroup holds, in an order that follows the schedule, so they agree to
rounding (1e-12 relative) and the best agents agree; the 512-thread
shape (two workgroups per CU) is also compared with the FP64 oracle
directly, with the same rounded couplings (1e-5 over 50 steps, as for the
default schedule)."""
import numpy as np
import pytest
import scipy.sparse as sp

import trackgen as tg
from oracle import ising as oising
from oracle import quant as oquant
from oracle import sb as osb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2402_14718_amd as sbt  # noqa: E402

# events from 20 to ~6000 variables: both shapes, several agents per item,
# rows past their slot's capacity
EVENTS = [(tg.tiny_spec(), 4), (tg.plain_spec(30), 1), (tg.plain_spec(150), 3),
          (tg.plain_spec(400), 5), (tg.plain_spec(700), 6), (tg.plain_spec(950), 7)]
TUNINGS = [dict(), dict(split_n=4608), dict(split_n=1152, fill=0.5), dict(fill=0.5, tail_words=4096),
           dict(split_n=4608, tail_words=0), dict(split_n=100000, fill=0.25, tail_words=2048)]


@pytest.fixture(scope="module")
def qubos():
    return [sbt.build_qubo(tg.generate(s, seed).hits_struct()) for s, seed in EVENTS]


def _run(qs, mode, prec, tuning, M=100, K=120, every=20):
    # aSB's explicit steps need a small dt (at dt = 1 these events diverge)
    dt = 0.1 if mode == "asb" else 1.0
    ds = sbt.DeviceBatchSolver(qs, mode, prec, sbt.solve_params(agents=M, steps=K, seed=9,
                                                               energy_every=every, dt=dt),
                               want_agent_energy=True, want_agent_state=True, want_trace=True,
                               tuning=sbt.batch_tuning(**tuning))
    ds.run()
    return ds.result(), ds.plan_info()


@pytest.mark.parametrize("mode,prec", [("dsb", "bf16"), ("bsb", "fp16"), ("asb", "bf16")])
def test_every_tuning_gives_bit_identical_results(qubos, mode, prec):
    assert max(q.n for q in qubos) > 4608 and min(q.n for q in qubos) < 100
    ref, info0 = _run(qubos, mode, prec, TUNINGS[0])
    assert all(np.all(np.isfinite(x)) for x in ref["agent_x"])
    items = {info0["work_items"]}
    for t in TUNINGS[1:]:
        r, info = _run(qubos, mode, prec, t)
        items.add(info["work_items"])
        for k in ("energy", "offset", "agent_energy", "trace", "agent_trace"):
            assert np.allclose(r[k], ref[k], rtol=1e-12, atol=1e-12), (t, k)
        assert np.array_equal(r["best_agent"], ref["best_agent"]), t
        for k in ("agent_x", "agent_T", "T"):
            assert all(np.array_equal(a, b) for a, b in zip(r[k], ref[k])), (t, k)
    assert len(items) > 1          # the tunings really schedule differently


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("mode", ["bsb", "dsb"])
def test_small_shape_trajectories_match_oracle(qubos, prec, mode):
    """Every event on the 512-thread shape, half-full items: 50 steps
    within 1e-5 of the oracle run with the same rounded couplings."""
    M, K, seed = 64, 50, 21
    qs = [q for q in qubos if q.n <= 4608]
    ds = sbt.DeviceBatchSolver(qs, mode, prec, sbt.solve_params(agents=M, steps=K, seed=seed),
                               want_agent_state=True,
                               tuning=sbt.batch_tuning(split_n=4608, fill=0.5))
    ds.run()
    r = ds.result()
    rnd = {"fp16": oquant.fp16_couplings, "bf16": oquant.bf16_couplings}[prec]
    for e, q in enumerate(qs):
        b = sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n))
        isg = oising.from_qubo(q.a, b)
        ref = osb.run(rnd(isg.J), isg.h, isg.c0, mode, M, K, seed=seed, event=e, margin_steps=K)
        x = r["agent_x"][e]
        err = np.linalg.norm(x - ref.x, axis=0) / np.linalg.norm(ref.x, axis=0)
        close = ref.wall_margin < 1e-6
        if mode == "dsb":
            close |= ref.sign_margin < 1e-6
        assert np.all((err <= 1e-5) | close), (e, err.max())
        assert np.mean(err <= 1e-5) >= 0.9


def test_cached_tuning_is_used_by_default(qubos):
    t = sbt.batch_tuning_lookup([q.n for q in qubos], "dsb", "bf16", 128)
    ds = sbt.DeviceBatchSolver(qubos, "dsb", "bf16", sbt.solve_params(agents=128, steps=10))
    assert sbt.tuning_dict(ds.tuning) == sbt.tuning_dict(t)
