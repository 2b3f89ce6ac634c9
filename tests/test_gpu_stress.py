"""Full-size parity on the stress event (5000 particles, N ~ 2.1e5, 512
agents, azimuth order): the GPU runs exactly the benchmark's launch
configuration; the FP64 oracle checks sampled rows.

After K steps row i depends only on the spins within K couplings of i, so
the oracle integrates the sub-problem induced by the 2-hop neighbourhood of
32 sampled rows, from the same Philox start and with the full problem's c0;
its x, y after two steps are exact for the sampled rows.  Energies of the
returned spins are checked for sampled agents on the whole QUBO."""
import numpy as np
import pytest
import scipy.sparse as sp

import trackgen as tg
from oracle import energy as oenergy
from oracle import ising as oising
from oracle import philox as ophilox
from oracle import quant as oquant
from oracle import sb as osb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2402_14718_amd as sbt  # noqa: E402

M, SEED = 512, 7


@pytest.fixture(scope="module")
def stress():
    ev = tg.generate(tg.stress_spec(), 300)
    hits = ev.hits_struct()
    bp = sbt.build_params_default()
    bp.z0_max = tg.STRESS_Z0_MAX
    q0 = sbt.build_qubo(hits, bp)
    q = sbt.permute_qubo(q0, sbt.phi_order(q0, hits))
    b = sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n))
    return q, b, oising.from_qubo(q.a, b)


def _two_hop(b, rows):
    s1 = np.union1d(rows, b[rows].indices)
    s2 = np.union1d(s1, b[s1].indices)
    return s1, s2


@pytest.mark.parametrize("prec", ["fp32", "fp8"])
@pytest.mark.parametrize("mode,kernel", [("bsb", "stream"), ("bsb", "stream_rows"),
                                         ("bsb", "stream_tile"), ("dsb", "stream")])
def test_two_steps_on_sampled_rows(stress, mode, kernel, prec):
    _sampled_rows_after_two_steps(stress, mode, kernel, prec)


@pytest.mark.parametrize("prec", ["fp8", "bf16x2", "fp32", "fp8_block", "bf16"])
def test_matrix_core_dsb_two_steps_on_sampled_rows(stress, prec):
    """The matrix-core dSB step in the benchmark's configuration (512
    agents: two sign words per wave; 13045 blocks of 16 rows)."""
    _sampled_rows_after_two_steps(stress, "dsb", "stream_mfma", prec)


def _sampled_rows_after_two_steps(stress, mode, kernel, prec):
    q, b, isg = stress
    K = 2
    r = sbt.solve(q, mode, agents=M, steps=K, seed=SEED, precision=prec, kernel=kernel,
                  want_state=True)
    assert r["kernel"] == kernel
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(q.n, 32, replace=False))
    s1, s2 = _two_hop(b, rows)
    assert s2.size < 60000
    # sub-problem on s2: the J rows of s1 are complete inside it
    J = isg.J[s2][:, s2].tocsr()
    if prec == "fp8":
        J, _, _ = oquant.fp8_rows(J)     # per-row scales of complete rows
    elif prec == "bf16x2":
        J = oquant.bf16x2_couplings(J)
    elif prec == "fp8_block":
        J = oquant.fp8_blocks(J)[0]      # blocks of 8 within complete rows
    elif prec == "bf16":
        J = oquant.bf16_couplings(J)
    x0, y0 = ophilox.initial_state(q.n, M, SEED, 0, spins=s2)
    ref = osb.run(J, isg.h[s2], isg.c0, mode, M, K, seed=SEED, x0=x0, y0=y0, margin_steps=K)
    pos = np.searchsorted(s2, rows)
    xr, xg = ref.x[pos], r["x"][rows].astype(np.float64)
    err = np.linalg.norm(xg - xr, axis=0) / np.maximum(np.linalg.norm(xr, axis=0), 1e-30)
    close = ref.wall_margin < 1e-6
    if mode == "dsb":
        close |= ref.sign_margin < 1e-6
    ok = err <= 1e-5
    assert np.all(ok | close), (err.max(), np.nonzero(~ok & ~close)[0][:5])
    assert np.mean(ok) >= 0.9
    yerr = np.abs(r["y"][rows] - ref.y[pos]).max(axis=0)
    assert np.all((yerr <= 1e-5) | close)


def test_full_length_energies_and_best(stress):
    """Bench configuration (bSB, FP8, 512 agents) at 400 steps: FP64
    energies of sampled agents against the oracle on the whole QUBO."""
    q, b, _ = stress
    r = sbt.solve(q, "bsb", agents=M, steps=400, seed=0, precision="fp8", want_state=True)
    assert r["kernel"] == "stream"
    T = (r["x"] >= 0).astype(np.int8)
    cols = np.array([0, 1, 63, 64, 255, 256, 511, r["best_agent"]])
    e_or = oenergy.qubo_energy(q.a, b, T[:, cols])
    assert np.allclose(r["agent_energy"][cols], e_or, rtol=1e-12, atol=1e-9)
    assert r["best_agent"] == int(np.argmin(r["agent_energy"]))
    assert np.array_equal(r["T"], T[:, r["best_agent"]])


@pytest.mark.parametrize("prec", ["fp32", "fp8"])
def test_tiled_step_equals_untiled_on_the_stress_event(stress, prec):
    """The stress event's tile plan: runs of up to 32 rows whose column
    unions fit the LDS capacity, and rows longer than it read from global
    memory; the untiled step's positions bit for bit."""
    q, _, _ = stress
    kw = dict(agents=M, steps=6, seed=SEED, precision=prec, want_state=True)
    a = sbt.solve(q, "bsb", kernel="stream", **kw)
    t = sbt.solve(q, "bsb", kernel="stream_tile", **kw)
    assert np.array_equal(a["x"], t["x"]) and np.array_equal(a["y"], t["y"])
    assert np.array_equal(a["agent_energy"], t["agent_energy"])


@pytest.mark.parametrize("prec", ["fp32", "fp8"])
def test_row_quad_step_equals_row_step_on_the_stress_event(stress, prec):
    """The bench configuration's streaming step (row quads, 512 agents)
    against the one-row-per-wave step on the stress event, bit for bit."""
    q, _, _ = stress
    kw = dict(agents=M, steps=6, seed=SEED, precision=prec, want_state=True)
    a = sbt.solve(q, "bsb", kernel="stream_rows", **kw)
    t = sbt.solve(q, "bsb", kernel="stream", **kw)
    assert np.array_equal(a["x"], t["x"]) and np.array_equal(a["y"], t["y"])
    assert np.array_equal(a["agent_energy"], t["agent_energy"])
