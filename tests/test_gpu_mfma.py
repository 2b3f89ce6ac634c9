"""GPU parity of the matrix-core dSB streaming step (SBT_KERNEL_STREAM_MFMA)
through the C ABI, against the FP64 oracle run with the same rounded
couplings (FP8 with one scale per row, BF16 hi + lo pairs: oracle.quant).

The step's products J_ij * sgn(x_j) are exact in the instruction; its FP32
sums are added in the instruction's order, so trajectories are held to the
same bar as the CSR step's: 1e-5 relative per agent over the run, close
calls (sign or wall margin under 1e-6 in the oracle) exempt, at least 90%
of agents within it.  Energies are FP64 of the true QUBO.  Shapes cover one
and two 64-agent sign words per wave, ragged agent counts, partial last
blocks of 16 rows, rows much longer than one K-step of 32 listed columns,
empty rows and a single spin.  FP32 couplings run as three exact BF16
terms, and so do block-scaled FP8 couplings, from their FP32 values;
BF16 and FP16 couplings (the batch functions' forms) are one operand."""
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

# FP32: the oracle keeps FP64 couplings (the kernel's FP32 rounding of J is
# inside the bar, as for every FP32 path)
FORMS = {"fp8": lambda J: oquant.fp8_rows(J)[0], "bf16x2": oquant.bf16x2_couplings,
         "fp32": lambda J: J, "fp8_block": lambda J: oquant.fp8_blocks(J)[0],
         "bf16": oquant.bf16_couplings, "fp16": oquant.fp16_couplings}


def _random_qubo(n, rows_deg, seed, empty=()):
    """Symmetric random QUBO: row i links to rows_deg(i) random others;
    rows in `empty` keep no coupling at all."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    keep = np.setdiff1d(np.arange(n), np.asarray(empty, dtype=np.int64))
    for i in keep:
        d = min(rows_deg(i), keep.size - 1)
        js = rng.choice(keep[keep != i], d, replace=False) if d > 0 else []
        rows += [i] * len(js)
        cols += list(js)
    B = sp.coo_matrix((rng.uniform(-1, 1, len(rows)), (rows, cols)), shape=(n, n)).tocsr()
    B = sp.triu(B + B.T, k=1)
    B = (B + B.T).tocsr()
    B.sort_indices()
    return sbt.Qubo(n, rng.uniform(0, 0.7, n), B.indptr.astype(np.int64), B.indices.astype(np.int32),
                    B.data.astype(np.float64), np.zeros((n, 3), np.int64))


def _random_qubo_large(n, deg, seed):
    """Symmetric random QUBO, about 2 deg couplings per row (vectorised)."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), deg)
    cols = rng.integers(0, n, rows.size)
    keep = rows != cols
    B = sp.coo_matrix((rng.uniform(-1, 1, int(keep.sum())), (rows[keep], cols[keep])),
                      shape=(n, n)).tocsr()
    B = sp.triu(B + B.T, k=1)
    B = (B + B.T).tocsr()
    B.sort_indices()
    return sbt.Qubo(n, rng.uniform(0, 0.7, n), B.indptr.astype(np.int64), B.indices.astype(np.int32),
                    B.data.astype(np.float64), np.zeros((n, 3), np.int64))


def _qubos():
    plain = sbt.build_qubo(tg.generate(tg.plain_spec(), 100).hits_struct())   # n = 1480
    # rows 0-9 link to 300 others (about ten K-steps per block), the rest 3;
    # rows 40-47 and the last 5 rows empty; n = 1013 (partial last block)
    dense = _random_qubo(1013, lambda i: 300 if i < 10 else 3, 3,
                         empty=list(range(40, 48)) + list(range(1008, 1013)))
    return {"plain": plain, "dense": dense}


QUBOS = _qubos()


def _check(q, prec, M, K, dt, seed):
    b = sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n))
    isg = oising.from_qubo(q.a, b)
    r = sbt.solve(q, "dsb", agents=M, steps=K, dt=dt, seed=seed, precision=prec,
                  kernel="stream_mfma", want_state=True)
    assert r["kernel"] == "stream_mfma"
    ref = osb.run(FORMS[prec](isg.J), isg.h, isg.c0, "dsb", M, K, dt=dt, seed=seed, margin_steps=K)
    err = np.linalg.norm(r["x"] - ref.x, axis=0) / np.maximum(np.linalg.norm(ref.x, axis=0), 1e-30)
    close = (ref.wall_margin < 1e-6) | (ref.sign_margin < 1e-6)
    ok = err <= 1e-5
    assert np.all(ok | close), (err.max(), np.nonzero(~ok & ~close)[0][:5])
    assert np.mean(ok) >= 0.9
    T = (r["x"] >= 0).astype(np.int8)
    e_or = oenergy.qubo_energy(q.a, b, T)
    assert np.all(np.abs(r["agent_energy"] - e_or) <= 1e-9 * np.maximum(1.0, np.abs(e_or)))
    return r


@pytest.mark.parametrize("prec", ["fp8", "bf16x2", "fp32", "fp8_block", "bf16", "fp16"])
@pytest.mark.parametrize("name", ["plain", "dense"])
@pytest.mark.parametrize("dt,K,M", [(1.0, 50, 70), (0.1, 20, 96), (0.1, 10, 600), (0.1, 20, 130),
                                    (0.1, 20, 40), (1.0, 30, 64), (0.1, 10, 1)])
def test_matrix_core_dsb_trajectory_within_1e5(prec, name, dt, K, M):
    """dt = 1 puts positions on the walls within ten steps; dt = 0.1 keeps
    them inside, where every coupling's arithmetic shows.  M = 40, 64 and 1
    run one sign word per wave, the others two (70, 130: partial words and
    tiles; 600: five agent groups)."""
    _check(QUBOS[name], prec, M, K, dt, seed=11)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 33])
def test_matrix_core_dsb_tiny_problems(n):
    """One spin (no coupling at all: F = h), one partial block, one exact
    block, a block and one row, two blocks and one row."""
    q = _random_qubo(n, lambda i: 4, 7)
    _check(q, "fp8", 70, 20, 0.1, seed=5)


def test_matrix_core_dsb_moves_with_the_coupling_form():
    """Inside the walls the BF16 pairs and the FP8 codes give measurably
    different trajectories (the forms are not silently swapped)."""
    q = QUBOS["plain"]
    kw = dict(agents=96, steps=10, dt=0.1, seed=2, kernel="stream_mfma", want_state=True)
    a = sbt.solve(q, "dsb", precision="fp8", **kw)
    c = sbt.solve(q, "dsb", precision="bf16x2", **kw)
    assert np.linalg.norm(a["x"] - c["x"]) > 1e-5 * np.linalg.norm(c["x"])


def test_matrix_core_dsb_full_length_quality():
    """5000 steps, 256 agents on the plain event: the best energy is within
    0.5% of the CSR step's on the same coupling form (over thousands of
    steps the rounding of the sums can send an agent another way), and the
    checkpoint trace is a best-so-far: non-increasing, its last entry the
    lower of the final best and the previous checkpoint."""
    q = QUBOS["plain"]
    kw = dict(agents=256, steps=5000, seed=1, precision="fp8", energy_every=500, want_trace=True)
    a = sbt.solve(q, "dsb", kernel="stream_mfma", **kw)
    c = sbt.solve(q, "dsb", kernel="stream", **kw)
    assert a["kernel"] == "stream_mfma" and c["kernel"] == "stream"
    assert a["energy"] <= c["energy"] + 0.005 * abs(c["energy"])
    tr = a["trace"]
    assert tr.shape == (10,) and np.all(np.diff(tr) <= 0)
    assert abs(tr[-1] - min(a["energy"], tr[-2])) <= 1e-9 * abs(tr[-1])


@pytest.mark.parametrize("prec", ["bf16x2", "fp32"])
def test_matrix_core_streamed_state_with_a_partial_agent_group(prec):
    """A state larger than the Infinity Cache (66000 spins x 520 agents,
    274.6 MB of x, y) takes the streamed path, where workgroups share the
    wide operands across four agent groups; 520 agents are five groups, so
    the second workgroup of every block has three idle waves.  Two steps on
    32 sampled rows against the oracle on their 2-hop neighbourhood (from
    the same Philox start), as on the stress event."""
    n, M, K, seed = 66000, 520, 2, 9
    q = _random_qubo_large(n, 2, 21)
    assert 8 * n * M > 256 << 20
    b = sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(n, n))
    isg = oising.from_qubo(q.a, b)
    r = sbt.solve(q, "dsb", agents=M, steps=K, seed=seed, precision=prec, kernel="stream_mfma",
                  want_state=True)
    rows = np.sort(np.random.default_rng(4).choice(n, 32, replace=False))
    s1 = np.union1d(rows, b[rows].indices)
    s2 = np.union1d(s1, b[s1].indices)
    J = FORMS[prec](isg.J[s2][:, s2].tocsr())
    x0, y0 = ophilox.initial_state(n, M, seed, 0, spins=s2)
    ref = osb.run(J, isg.h[s2], isg.c0, "dsb", M, K, seed=seed, x0=x0, y0=y0, margin_steps=K)
    pos = np.searchsorted(s2, rows)
    xr, xg = ref.x[pos], r["x"][rows].astype(np.float64)
    err = np.linalg.norm(xg - xr, axis=0) / np.maximum(np.linalg.norm(xr, axis=0), 1e-30)
    close = (ref.wall_margin < 1e-6) | (ref.sign_margin < 1e-6)
    ok = err <= 1e-5
    assert np.all(ok | close), (err.max(), np.nonzero(~ok & ~close)[0][:5])
    assert np.mean(ok) >= 0.9


@pytest.mark.parametrize("mode,prec", [("bsb", "fp8"), ("asb", "bf16x2"), ("bsb", "fp32"),
                                       ("asb", "fp8_block")])
def test_matrix_core_step_refuses_other_modes_and_forms(mode, prec):
    q = sbt.build_qubo(tg.generate(tg.plain_spec(60), 2).hits_struct())
    with pytest.raises(sbt.SbtError) as e:
        sbt.solve(q, mode, agents=64, steps=4, precision=prec, kernel="stream_mfma")
    assert e.value.code == -4
