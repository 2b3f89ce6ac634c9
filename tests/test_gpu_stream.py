"""GPU parity of the streaming step kernel (one launch per step, state in
HBM) and of its FP8 coupling form, through the C ABI, against the oracle.

FP8: the oracle runs with the same per-row E4M3 couplings
(``oracle.quant.fp8_rows``), everything else in FP64, so the FP32
trajectories must stay within 1e-5 relative over 50 steps, with the same
close-call allowance as the FP32 path.  Energies are of the true QUBO, FP64.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import trackgen as tg
from oracle import energy as oenergy
from oracle import ising as oising
from oracle import quant as oquant
from oracle import sb as osb
from oracle import tracks as otracks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2402_14718_amd as sbt  # noqa: E402
from paper_2402_14718_amd import _lib  # noqa: E402


def _event(spec, seed):
    ev = tg.generate(spec, seed)
    q = sbt.build_qubo(ev.hits_struct())
    b = sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n))
    return ev, q, b, oising.from_qubo(q.a, b)


@pytest.mark.parametrize("mode", ["bsb", "dsb"])
@pytest.mark.parametrize("dt,K", [(1.0, 50), (0.1, 10), (0.1, 20)])
def test_fp8_trajectory_within_1e5(mode, dt, K):
    """dt = 1 puts every position of this event on the wall within ten steps;
    dt = 0.1 keeps the state inside (all of it at K = 10, about a quarter at
    K = 20), where the arithmetic of every coupling shows."""
    ev, q, b, isg = _event(tg.plain_spec(), 100)
    Jq, codes, scale = oquant.fp8_rows(isg.J)
    M, seed = 70, 11                          # 70 agents: a ragged second 64-agent word
    r = sbt.solve(q, mode, agents=M, steps=K, dt=dt, seed=seed, precision="fp8", want_state=True)
    assert r["kernel"] == "stream"
    ref = osb.run(Jq, isg.h, isg.c0, mode, M, K, dt=dt, seed=seed, margin_steps=K)
    err = np.linalg.norm(r["x"] - ref.x, axis=0) / np.linalg.norm(ref.x, axis=0)
    close_call = ref.wall_margin < 1e-6
    if mode == "dsb":
        close_call |= ref.sign_margin < 1e-6
    ok = err <= 1e-5
    assert np.all(ok | close_call), (err.max(), np.nonzero(~ok & ~close_call))
    assert np.mean(ok) >= 0.9
    if dt < 1.0:
        # inside the walls the FP8 couplings move the state measurably away
        # from the FP32 ones (about 3e-4 relative at K = 10)
        r32 = sbt.solve(q, mode, agents=M, steps=K, dt=dt, seed=seed, kernel="stream",
                        want_state=True)
        assert np.linalg.norm(r32["x"] - r["x"]) > 1e-5 * np.linalg.norm(r["x"])


@pytest.mark.parametrize("mode", ["bsb", "dsb"])
def test_fp8_energies_are_exact_fp64_of_the_true_qubo(mode):
    ev, q, b, isg = _event(tg.plain_spec(), 101)
    r = sbt.solve(q, mode, agents=96, steps=800, seed=2, precision="fp8", want_state=True)
    T = (r["x"] >= 0).astype(np.int8)
    e_or = oenergy.qubo_energy(q.a, b, T)
    assert np.all(np.abs(r["agent_energy"] - e_or) <= 1e-9 * np.maximum(1.0, np.abs(e_or)))
    best = oenergy.best_agent(e_or)
    assert r["best_agent"] == best and np.array_equal(r["T"], T[:, best])


def test_fp8_rejected_on_resident_kernel_and_16_bit_single_event():
    ev, q, b, isg = _event(tg.tiny_spec(), 1)
    with pytest.raises(sbt.SbtError) as e:
        sbt.solve(q, "dsb", agents=8, steps=10, precision="fp8", kernel="resident")
    assert e.value.code == _lib.SBT_EUNSUPPORTED
    with pytest.raises(sbt.SbtError) as e:
        sbt.solve(q, "dsb", agents=8, steps=10, precision="fp16")
    assert e.value.code == _lib.SBT_EUNSUPPORTED


@pytest.mark.parametrize("mode", ["bsb", "dsb"])
def test_fp8_full_size_quality(mode):
    """Plain workload at full length: the FP8 form's best energy within 0.5%
    of the FP32 solver's best over the same agents, efficiency and purity
    within 0.02."""
    ev, q, b, isg = _event(tg.plain_spec(), 100)
    r8 = sbt.solve(q, mode, agents=256, steps=5000, seed=0, precision="fp8")
    r32 = sbt.solve(q, mode, agents=256, steps=5000, seed=0)
    assert r8["energy"] <= r32["energy"] + 0.005 * abs(r32["energy"])
    eff8, pur8, *_ = otracks.evaluate(ev, q.trip_hits, r8["T"])
    eff32, pur32, *_ = otracks.evaluate(ev, q.trip_hits, r32["T"])
    assert abs(eff8 - eff32) <= 0.02 and abs(pur8 - pur32) <= 0.02


@pytest.mark.parametrize("M", [1, 63, 64, 65, 130, 600, 1100, 1101])
def test_stream_agent_words_ragged(M):
    """Agent counts around the 64-agent word of the sign planes and past one
    wave's 512 (dSB) / 256 (bSB) agents -- several agent blocks per row, a
    ragged last block, the four-agents-per-lane bSB variant (M % 4 = 0) and
    the lane-strided one: the streaming kernel against the resident one, bit
    for bit."""
    ev, q, b, isg = _event(tg.plain_spec(60), 7)
    for mode in ("bsb", "dsb"):
        rr = sbt.solve(q, mode, agents=M, steps=120, seed=9, kernel="resident", want_state=True)
        rs = sbt.solve(q, mode, agents=M, steps=120, seed=9, kernel="stream", want_state=True)
        assert np.array_equal(rr["x"], rs["x"]), mode
        assert np.array_equal(rr["y"], rs["y"]), mode


@pytest.mark.parametrize("prec", ["fp32", "fp8"])
@pytest.mark.parametrize("M", [70, 96])
def test_asb_trajectory_matches_oracle(prec, M):
    """aSB (Eq. 1-2, no walls) on the streaming kernel; dt = 0.1 (its
    explicit steps diverge on this event at dt >= 0.5).  M = 96 runs the
    four-agents-per-lane variant, M = 70 the lane-strided one."""
    ev, q, b, isg = _event(tg.plain_spec(), 100)
    J = oquant.fp8_rows(isg.J)[0] if prec == "fp8" else isg.J
    K, dt, seed = 20, 0.1, 11
    r = sbt.solve(q, "asb", agents=M, steps=K, dt=dt, seed=seed, precision=prec, kernel="stream",
                  want_state=True)
    assert r["kernel"] == "stream"
    ref = osb.run(J, isg.h, isg.c0, "asb", M, K, dt=dt, seed=seed)
    err = np.linalg.norm(r["x"] - ref.x, axis=0) / np.linalg.norm(ref.x, axis=0)
    assert np.all(err <= 1e-5), err.max()
    assert np.abs(ref.x).max() > 1.0            # no wall: positions leave [-1, 1]
    yerr = np.linalg.norm(r["y"] - ref.y, axis=0) / np.linalg.norm(ref.y, axis=0)
    assert np.all(yerr <= 1e-5), yerr.max()


def test_asb_energies_and_every_kernel():
    """aSB energies are the FP64 QUBO objective of the returned spins; the
    resident kernel runs the same steps bit for bit."""
    ev, q, b, isg = _event(tg.plain_spec(), 101)
    r = sbt.solve(q, "asb", agents=64, steps=300, dt=0.1, seed=2, kernel="stream", want_state=True)
    T = (r["x"] >= 0).astype(np.int8)
    e_or = oenergy.qubo_energy(q.a, b, T)
    assert np.all(np.abs(r["agent_energy"] - e_or) <= 1e-9 * np.maximum(1.0, np.abs(e_or)))
    rr = sbt.solve(q, "asb", agents=64, steps=300, dt=0.1, seed=2, kernel="resident",
                   want_state=True)
    assert r["kernel"] == "stream" and rr["kernel"] == "resident"
    assert np.array_equal(rr["x"], r["x"]) and np.array_equal(rr["y"], r["y"])
    with pytest.raises(sbt.SbtError) as e:
        sbt.solve(q, "asb", agents=8, steps=10, precision="fp8", kernel="resident")
    assert e.value.code == _lib.SBT_EUNSUPPORTED


def _dense_rows_qubo(n=1500, dense=10, deg=700, seed=3):
    """Random symmetric QUBO whose first `dense` rows couple to `deg` others:
    rows longer than a tile's column capacity (tiles of their own, read from
    global memory) beside short rows."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(dense):
        js = rng.choice(np.arange(dense, n), deg, replace=False)
        rows += [i] * deg
        cols += list(js)
    for i in range(dense, n):
        js = rng.choice(n, 3, replace=False)
        rows += [i] * 3
        cols += list(js)
    B = sp.coo_matrix((rng.uniform(-1, 1, len(rows)), (rows, cols)), shape=(n, n)).tocsr()
    B = sp.triu(B + B.T, k=1)
    B = (B + B.T).tocsr()
    B.sort_indices()
    return sbt.Qubo(n, rng.uniform(0, 0.7, n), B.indptr.astype(np.int64),
                    B.indices.astype(np.int32), B.data.astype(np.float64),
                    np.zeros((n, 3), np.int64))


@pytest.mark.parametrize("mode", ["bsb", "asb"])
@pytest.mark.parametrize("prec", ["fp32", "fp8", "fp8_block", "bf16x2"])
@pytest.mark.parametrize("M", [64, 96, 130, 600])
def test_tiled_step_bit_identical_to_untiled(mode, prec, M):
    """The tiled streaming step (planned row tiles, column unions in LDS)
    against the untiled one: plain event (tiles of several rows), a QUBO
    with rows longer than a tile holds (read from global memory) between
    short ones; ragged agent counts (partial 64-agent blocks; 130 agents
    stage one agent per load, the others four)."""
    dt = 0.1 if mode == "asb" else 1.0
    for q in (sbt.build_qubo(tg.generate(tg.plain_spec(), 104).hits_struct()), _dense_rows_qubo()):
        kw = dict(agents=M, steps=40, seed=3, dt=dt, precision=prec, want_state=True)
        a = sbt.solve(q, mode, kernel="stream", **kw)
        t = sbt.solve(q, mode, kernel="stream_tile", **kw)
        assert t["kernel"] == "stream_tile"
        assert np.array_equal(a["x"], t["x"]) and np.array_equal(a["y"], t["y"])
        assert np.array_equal(a["agent_energy"], t["agent_energy"])


def test_tiled_step_refuses_dsb():
    q = sbt.build_qubo(tg.generate(tg.plain_spec(60), 2).hits_struct())
    with pytest.raises(sbt.SbtError) as e:
        sbt.solve(q, "dsb", agents=64, steps=4, kernel="stream_tile")
    assert e.value.code == -4


FORMS = {"fp8_block": lambda J: oquant.fp8_blocks(J)[0], "bf16x2": oquant.bf16x2_couplings}


@pytest.mark.parametrize("prec", ["fp8_block", "bf16x2"])
@pytest.mark.parametrize("mode", ["bsb", "dsb"])
@pytest.mark.parametrize("dt,K,M", [(1.0, 50, 70), (0.1, 20, 96), (0.1, 10, 600)])
def test_block_fp8_and_bf16_pair_trajectories_within_1e5(prec, mode, dt, K, M):
    """FP8 with a scale per block of eight couplings and BF16 hi + lo pairs
    on the streaming kernel against the oracle run with the same rounded
    couplings (oracle.quant): 1e-5 per agent, close calls exempt, >= 90%
    of agents; FP64 energies of the returned spins exact."""
    ev, q, b, isg = _event(tg.plain_spec(), 100)
    Jq = FORMS[prec](isg.J)
    r = sbt.solve(q, mode, agents=M, steps=K, dt=dt, seed=11, precision=prec, want_state=True)
    assert r["kernel"] == "stream"
    ref = osb.run(Jq, isg.h, isg.c0, mode, M, K, dt=dt, seed=11, margin_steps=K)
    err = np.linalg.norm(r["x"] - ref.x, axis=0) / np.linalg.norm(ref.x, axis=0)
    close = ref.wall_margin < 1e-6
    if mode == "dsb":
        close |= ref.sign_margin < 1e-6
    ok = err <= 1e-5
    assert np.all(ok | close), (err.max(), np.nonzero(~ok & ~close))
    assert np.mean(ok) >= 0.9
    T = (r["x"] >= 0).astype(np.int8)
    e_or = oenergy.qubo_energy(q.a, b, T)
    assert np.all(np.abs(r["agent_energy"] - e_or) <= 1e-9 * np.maximum(1.0, np.abs(e_or)))


def test_new_forms_refused_where_not_built():
    q = sbt.build_qubo(tg.generate(tg.plain_spec(60), 2).hits_struct())
    for prec in ("fp8_block", "bf16x2"):
        with pytest.raises(sbt.SbtError) as e:
            sbt.solve(q, "bsb", agents=8, steps=4, precision=prec, kernel="resident")
        assert e.value.code == -4


def _tile_edge_qubo(seed=5):
    """A QUBO built to hit the tile plan's limits: seven rows sharing one set
    of 90 neighbours (96 padded couplings each, so the 640-coupling bound
    closes a tile after six of them while the union is still small), rows
    of exactly 192 padded couplings (a tile's whole column capacity), a row
    of 200 (past it: read from global memory), sparse rows elsewhere, and
    n = 1013 (a partial last block of 32 rows)."""
    rng = np.random.default_rng(seed)
    n = 1013
    rows, cols = [], []

    def link(i, js):
        rows.extend([i] * len(js))
        cols.extend(js)

    shared = list(range(500, 590))
    for i in range(7):
        link(i, shared)
    link(100, list(range(600, 792)))
    link(102, list(range(601, 793)))
    link(101, list(range(600, 797)))
    for i in range(110, n):  # never touching the rows above
        link(i, list(110 + rng.choice(n - 110, 3, replace=False)))
    B = sp.coo_matrix((rng.uniform(-1, 1, len(rows)), (rows, cols)), shape=(n, n)).tocsr()
    B = sp.triu(B + B.T, k=1)
    B = (B + B.T).tocsr()
    B.sort_indices()
    return sbt.Qubo(n, rng.uniform(0, 0.7, n), B.indptr.astype(np.int64), B.indices.astype(np.int32),
                    B.data.astype(np.float64), np.zeros((n, 3), np.int64))


@pytest.mark.parametrize("M", [64, 130])
@pytest.mark.parametrize("prec", ["fp32", "fp8_block"])
def test_tiled_step_at_the_tile_limits(M, prec):
    q = _tile_edge_qubo()
    lens = np.diff(q.row_ptr)
    plen = (lens + 7) // 8 * 8
    assert np.all(plen[:7] == 96) and plen[100] == 192 and plen[102] == 192 and plen[101] == 200
    kw = dict(agents=M, steps=30, seed=4, precision=prec, want_state=True)
    a = sbt.solve(q, "bsb", kernel="stream", **kw)
    t = sbt.solve(q, "bsb", kernel="stream_tile", **kw)
    assert np.array_equal(a["x"], t["x"]) and np.array_equal(a["y"], t["y"])
    assert np.array_equal(a["agent_energy"], t["agent_energy"])


@pytest.mark.parametrize("mode", ["bsb", "asb"])
@pytest.mark.parametrize("prec", ["fp32", "fp8", "fp8_block", "bf16x2"])
@pytest.mark.parametrize("M", [68, 260, 600])
def test_row_quad_step_bit_identical_to_row_step(mode, prec, M):
    """The streaming step over row quads (each distinct neighbour of four
    rows gathered once) against the one-row-per-wave step: plain event, a
    QUBO with dense rows and empty rows, the tile-limit QUBO (n = 1013, a
    partial last quad); agent counts with a partial 256-agent block."""
    dt = 0.1 if mode == "asb" else 1.0
    for q in (sbt.build_qubo(tg.generate(tg.plain_spec(), 104).hits_struct()), _dense_rows_qubo(),
              _tile_edge_qubo()):
        kw = dict(agents=M, steps=40, seed=3, dt=dt, precision=prec, want_state=True)
        a = sbt.solve(q, mode, kernel="stream_rows", **kw)
        t = sbt.solve(q, mode, kernel="stream", **kw)
        assert a["kernel"] == "stream_rows" and t["kernel"] == "stream"
        assert np.array_equal(a["x"], t["x"]) and np.array_equal(a["y"], t["y"])
        assert np.array_equal(a["agent_energy"], t["agent_energy"])
