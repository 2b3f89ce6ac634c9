"""C-ABI checks that need no GPU: symbols, host QUBO construction parity
with the oracle (bit-exact), host FP64 energy, and argument validation."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import trackgen as tg
from oracle import energy as oenergy
from oracle import qubo as oqubo

sbt = pytest.importorskip("paper_2402_14718_amd")
from paper_2402_14718_amd import _lib  # noqa: E402

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "sbtrack.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbt_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = sbt.load()
    names = _declared_functions()
    assert "sbt_solve" in names and "sbt_build_qubo" in names and "sbt_solve_dev" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(n for n, _, _ in _lib.EXPORTS) == set(names)


def test_struct_sizes_match_c_layout():
    assert C.sizeof(_lib.SbtHit) == 40
    assert C.sizeof(_lib.SbtBuildParams) == 6 * 8 + 2 * 4 + 4 * 8
    assert C.sizeof(_lib.SbtSolveParams) == 3 * 8 + 2 * 4 + 8 + 6 * 4
    assert sbt.HIT_DTYPE.itemsize == C.sizeof(_lib.SbtHit)


def test_default_params_match_oracle():
    p = sbt.build_params_default()
    o = oqubo.BuildParams()
    assert p.dphi_tan == o.dphi_tan and p.dtheta_tan == o.dtheta_tan
    assert (p.curv_max, p.dcurv_max, p.s_min) == (o.curv_max, o.dcurv_max, o.s_min)
    assert (p.max_holes, p.min_track_hits) == (o.max_holes, o.min_track_hits)
    assert (p.alpha, p.beta, p.gamma_, p.lambda_) == (o.alpha, o.beta, o.gamma, o.lam)


@pytest.mark.parametrize("spec,seed", [
    (tg.tiny_spec(), 1), (tg.tiny_spec(), 7), (tg.plain_spec(), 100), (tg.plain_spec(), 103),
    (tg.plain_spec(120), 5), (tg.EventSpec(n_particles=300, eta_max=0.6, noise_frac=0.3), 9),
])
def test_build_qubo_bit_exact_with_oracle(spec, seed):
    ev = tg.generate(spec, seed)
    q = sbt.build_qubo(ev.hits_struct())
    o = oqubo.build_event(ev)
    assert q.n == o.n
    assert np.array_equal(q.trip_hits, o.trip_hits)
    assert np.array_equal(q.row_ptr, o.b.indptr)
    assert np.array_equal(q.col, o.b.indices)
    assert np.array_equal(q.b, o.b.data)
    assert np.array_equal(q.a, o.a)


def test_build_qubo_orders_by_hit_id_not_input_order():
    ev = tg.generate(tg.plain_spec(80), 2)
    hits = ev.hits_struct()
    perm = np.random.default_rng(0).permutation(hits.shape[0])
    q1 = sbt.build_qubo(hits)
    q2 = sbt.build_qubo(hits[perm])
    assert np.array_equal(q1.trip_hits, q2.trip_hits)
    assert np.array_equal(q1.b, q2.b) and np.array_equal(q1.a, q2.a)


def test_build_qubo_params_and_edge_cases():
    ev = tg.generate(tg.tiny_spec(), 3)
    hits = ev.hits_struct()
    p = sbt.build_params_default()
    p.min_track_hits = 5                      # four layers cannot make five hits
    assert sbt.build_qubo(hits, p).n == 0
    p.min_track_hits = 6
    with pytest.raises(sbt.SbtError) as e:
        sbt.build_qubo(hits, p)
    assert e.value.code == _lib.SBT_EUNSUPPORTED
    assert sbt.build_qubo(hits[:0]).n == 0       # no hits: empty QUBO
    bad = hits.copy()
    bad["x"][3] = np.nan
    with pytest.raises(sbt.SbtError) as e:
        sbt.build_qubo(bad)
    assert e.value.code == _lib.SBT_EINVAL
    dup = hits.copy()
    dup["hit_id"][5] = dup["hit_id"][4]
    with pytest.raises(sbt.SbtError):
        sbt.build_qubo(dup)


def test_host_energy_matches_oracle():
    ev = tg.generate(tg.plain_spec(), 101)
    q = sbt.build_qubo(ev.hits_struct())
    o = oqubo.build_event(ev)
    rng = np.random.default_rng(4)
    for _ in range(5):
        T = (rng.random(q.n) < 0.5).astype(np.int8)
        e_lib = sbt.energy(q, T)
        e_or = float(oenergy.qubo_energy(o.a, o.b, T))
        assert abs(e_lib - e_or) <= 1e-12 * max(1.0, abs(e_or))
    with pytest.raises(sbt.SbtError):
        sbt.energy(q, np.full(q.n, 2, dtype=np.int8))


def test_workspace_and_param_validation():
    p = sbt.solve_params(agents=256, steps=5000)
    ws = sbt.workspace_bytes(1500, 3000, "bsb", p)
    assert ws >= 3 * 1500 * 256 * 4                 # x ping-pong + y
    for bad in [dict(agents=0), dict(steps=0), dict(dt=0.0), dict(a0=-1.0), dict(energy_every=-1)]:
        kw = dict(agents=8, steps=10)
        kw.update(bad)
        with pytest.raises(sbt.SbtError):
            sbt.workspace_bytes(100, 200, "dsb", sbt.solve_params(**kw))
    with pytest.raises(sbt.SbtError):
        sbt.workspace_bytes(0, 0, "dsb", sbt.solve_params())
    with pytest.raises(sbt.SbtError):
        sbt.workspace_bytes(1 << 20, 0, "dsb", sbt.solve_params(agents=4096))
    # dSB updates x in place: one position buffer plus two sign planes
    wd = sbt.workspace_bytes(1500, 3000, "dsb", p)
    assert 2 * 1500 * 256 * 4 + 2 * 1500 * 4 * 8 <= wd < ws
    # FP8 adds one byte per padded coupling and a scale per row
    w8 = sbt.workspace_bytes(1500, 3000, "bsb", sbt.solve_params(agents=256, steps=5000,
                                                                precision="fp8"))
    assert w8 >= ws + 3000 + 1500 * 4


def test_precision_selects_or_rejects_kernels():
    n, nnz, row = 1480, 2722, 12
    # FP32: either kernel, depending on the device's LDS size
    assert sbt.select_kernel(n, nnz, row, "dsb", sbt.solve_params(agents=256)) in ("resident",
                                                                                 "stream")
    assert sbt.select_kernel(n, nnz, row, "dsb",
                             sbt.solve_params(agents=256, precision="fp8")) == "stream"
    with pytest.raises(sbt.SbtError) as e:
        sbt.select_kernel(n, nnz, row, "dsb",
                          sbt.solve_params(agents=256, precision="fp8", kernel="resident"))
    assert e.value.code == _lib.SBT_EUNSUPPORTED
    for prec in ("fp16", "bf16"):
        with pytest.raises(sbt.SbtError) as e:
            sbt.select_kernel(n, nnz, row, "bsb", sbt.solve_params(precision=prec))
        assert e.value.code == _lib.SBT_EUNSUPPORTED
    p = sbt.solve_params()
    p.precision = 9
    with pytest.raises(sbt.SbtError) as e:
        sbt.select_kernel(n, nnz, row, "bsb", p)
    assert e.value.code == _lib.SBT_EINVAL
    p = sbt.solve_params()
    p.reserved = 1
    with pytest.raises(sbt.SbtError):
        sbt.select_kernel(n, nnz, row, "bsb", p)


def test_matrix_core_step_selection_and_workspace():
    """The matrix-core step runs on request only, for dSB with FP8 (per-row
    scale) or BF16X2 couplings; its block lists and operand tiles add at
    most (nnz / 32 + n / 16 + 1) K-steps of 640 (FP8) or 2176 (BF16X2)
    bytes, x and y in its tiles (rows padded to 16, agents to 128) two
    more copies of the state, and its sign records replace the sign
    words."""
    n, nnz, row = 1480, 2722, 12
    for prec in ("fp8", "bf16x2", "fp32", "fp8_block", "bf16", "fp16"):
        p = sbt.solve_params(agents=256, precision=prec, kernel="stream_mfma")
        assert sbt.select_kernel(n, nnz, row, "dsb", p) == "stream_mfma"
        if prec in ("bf16", "fp16"):   # below the threshold: the batch functions' forms
            with pytest.raises(sbt.SbtError) as e:
                sbt.select_kernel(n, nnz, row, "dsb", sbt.solve_params(agents=256, precision=prec))
            assert e.value.code == _lib.SBT_EUNSUPPORTED
            continue
        assert sbt.select_kernel(n, nnz, row, "dsb", sbt.solve_params(agents=256, precision=prec)) \
            in (("stream", "resident") if prec == "fp32" else ("stream",))
        # AUTO: the matrix-core step from 2^23 spin-agent pairs on (the stress
        # event, 208710 x 512; the precision event, 8493 x 1024), the CSR
        # step just below and for bSB
        big = sbt.solve_params(agents=512, precision=prec)
        assert sbt.select_kernel(208710, 11248462, 73, "dsb", big) == "stream_mfma"
        assert sbt.select_kernel(8493, 30964, 12, "dsb",
                                 sbt.solve_params(agents=1024, precision=prec)) == "stream_mfma"
        assert sbt.select_kernel(16384, 60000, 12, "dsb", big) == "stream_mfma"   # 2^23 exactly
        assert sbt.select_kernel(16383, 60000, 12, "dsb", big) in ("stream", "resident")
        assert sbt.select_kernel(208710, 11248462, 73, "bsb", big) == "stream"
        assert sbt.select_kernel(208710, 11248462, 73, "dsb",
                                 sbt.solve_params(agents=512, precision=prec, kernel="stream")) \
            == "stream"
    assert sbt.select_kernel(n, nnz, row, "dsb", sbt.solve_params(agents=256, precision="fp32",
                                                                   kernel="stream_mfma")) == "stream_mfma"
    assert sbt.select_kernel(n, nnz, row, "dsb", sbt.solve_params(
        agents=256, precision="fp8_block", kernel="stream_mfma")) == "stream_mfma"
    for mode, prec in (("bsb", "fp8"), ("asb", "bf16x2"), ("bsb", "fp32"), ("asb", "fp8_block")):
        with pytest.raises(sbt.SbtError) as e:
            sbt.select_kernel(n, nnz, row, mode,
                              sbt.solve_params(agents=256, precision=prec, kernel="stream_mfma"))
        assert e.value.code == _lib.SBT_EUNSUPPORTED
    ks = nnz // 32 + (n + 15) // 16 + 1
    tiles = 2 * 4 * ((n + 15) // 16 * 16) * ((256 + 127) // 128 * 128)
    for prec, per in (("fp8", 640), ("bf16x2", 2176), ("fp32", 3200), ("fp8_block", 3200)):
        base = sbt.workspace_bytes(n, nnz, "dsb", sbt.solve_params(agents=256, precision=prec,
                                                                   kernel="stream"))
        mf = sbt.workspace_bytes(n, nnz, "dsb", sbt.solve_params(agents=256, precision=prec,
                                                                 kernel="stream_mfma"))
        assert base + ks * per + tiles <= mf <= base + ks * per + tiles + 4 * (n + 16) + 8 * 256


def test_solve_rejects_malformed_qubo_before_touching_a_device():
    ev = tg.generate(tg.plain_spec(60), 1)
    q = sbt.build_qubo(ev.hits_struct())
    asym = sbt.Qubo(q.n, q.a.copy(), q.row_ptr.copy(), q.col.copy(), q.b.copy(), q.trip_hits)
    asym.b[0] += 0.5
    with pytest.raises(sbt.SbtError) as e:
        sbt.solve(asym, "dsb", agents=4, steps=5)
    assert e.value.code == _lib.SBT_EINVAL and "symmetric" in str(e.value)
    empty = sbt.Qubo(0, np.zeros(0), np.zeros(1, np.int64), np.zeros(0, np.int32),
                     np.zeros(0), np.zeros((0, 3), np.int64))
    with pytest.raises(sbt.SbtError):
        sbt.solve(empty, "bsb", agents=4, steps=5)
    nanq = sbt.Qubo(q.n, q.a.copy(), q.row_ptr, q.col, q.b, q.trip_hits)
    nanq.a[0] = np.inf
    with pytest.raises(sbt.SbtError):
        sbt.solve(nanq, "bsb", agents=4, steps=5)


@pytest.mark.parametrize("spec,seed", [(tg.plain_spec(), 100), (tg.plain_spec(300), 3),
                                       (tg.tiny_spec(), 2)])
def test_phi_order_and_permutation_bit_exact_with_oracle(spec, seed):
    from oracle import order as oorder
    ev = tg.generate(spec, seed)
    hits = ev.hits_struct()
    q = sbt.build_qubo(hits)
    perm = sbt.phi_order(q, hits[::-1])           # hit order must not matter
    o = oorder.phi_order(q.trip_hits, ev.hit_id, ev.x, ev.y, ev.z)
    assert np.array_equal(perm, o)
    qp = sbt.permute_qubo(q, perm)
    import scipy.sparse as sp
    a2, b2, th2 = oorder.permute(q.a, sp.csr_matrix((q.b, q.col, q.row_ptr), shape=(q.n, q.n)),
                                 q.trip_hits, o)
    assert np.array_equal(qp.a, a2) and np.array_equal(qp.trip_hits, th2)
    assert np.array_equal(qp.row_ptr, b2.indptr) and np.array_equal(qp.col, b2.indices)
    assert np.array_equal(qp.b, b2.data)
    T = (np.random.default_rng(seed).random(q.n) < 0.4).astype(np.int8)
    assert abs(sbt.energy(qp, T[perm]) - sbt.energy(q, T)) <= 1e-12 * max(1.0, abs(sbt.energy(q, T)))


def test_permutation_rejects_bad_input():
    ev = tg.generate(tg.tiny_spec(), 1)
    hits = ev.hits_struct()
    q = sbt.build_qubo(hits)
    bad = np.arange(q.n, dtype=np.int32)
    bad[0] = bad[1]
    with pytest.raises(sbt.SbtError) as e:
        sbt.permute_qubo(q, bad)
    assert e.value.code == _lib.SBT_EINVAL
    with pytest.raises(sbt.SbtError) as e:
        sbt.phi_order(q, hits[:3])                # triplets name hits not given
    assert e.value.code == _lib.SBT_EINVAL


@pytest.mark.parametrize("row_ptr,nnz", [([0, 10, 5], 5), ([0, 3, 1, 4], 4), ([0, -2, 4], 4)])
def test_malformed_row_pointers_rejected_before_rows_are_read(row_ptr, nnz):
    """A row_ptr that decreases or leaves [0, nnz] between its two ends is
    refused (SBT_EINVAL) by the single, batch and c0-scan entry points
    before any row is walked."""
    n = len(row_ptr) - 1
    q = sbt.Qubo(n, np.zeros(n), np.array(row_ptr, np.int64),
                 np.zeros(nnz, np.int32), np.zeros(nnz), np.zeros((n, 3), np.int64))
    with pytest.raises(sbt.SbtError) as e:
        sbt.solve(q, "dsb", agents=4, steps=5)
    assert e.value.code == _lib.SBT_EINVAL and "row_ptr" in str(e.value)
    with pytest.raises(sbt.SbtError) as e:
        sbt.solve_batch([q], "dsb", "fp16", agents=4, steps=5)
    assert e.value.code == _lib.SBT_EINVAL and "row_ptr" in str(e.value)
    with pytest.raises(sbt.SbtError) as e:
        sbt.c0_scan(q, "dsb", [1.0, 2.0], agents=4, steps=5)
    assert e.value.code == _lib.SBT_EINVAL and "row_ptr" in str(e.value)


def test_noalloc_entry_point_refuses_oversized_shapes_before_any_device_call():
    """sbt_solve_dev_noalloc checks the workspace this shape needs against
    its fixed array before touching a device (the pointers here are never
    read), and rejects invalid parameters the same way."""
    lib = sbt.load()
    fake = C.c_void_p(0x1000)
    dq = _lib.SbtDevQubo(1480, 2722, fake, fake, fake, fake)
    dr = _lib.SbtDevResult(fake, fake, fake, fake)
    p = sbt.solve_params(agents=8192, steps=100)
    need = sbt.workspace_bytes(1480, 2722, "bsb", p)
    assert need > 64 << 20
    rc = lib.sbt_solve_dev_noalloc(C.byref(dq), 12, _lib.SBT_BSB, C.byref(p), C.byref(dr), None)
    assert rc == _lib.SBT_EINVAL
    assert "limit" in lib.sbt_last_error().decode()
    p = sbt.solve_params(agents=0)
    rc = lib.sbt_solve_dev_noalloc(C.byref(dq), 12, _lib.SBT_BSB, C.byref(p), C.byref(dr), None)
    assert rc == _lib.SBT_EINVAL


def test_top_k_refuses_bad_sizes_before_any_device_call():
    """sbt_top_k_dev checks its sizes and pointers before launching (the
    pointers here are never read)."""
    lib = sbt.load()
    fake = C.c_void_p(0x1000)
    for agents, k in ((0, 1), (10, 0), (10, 11), (-3, 1)):
        assert lib.sbt_top_k_dev(fake, agents, k, fake, fake, None) == _lib.SBT_EINVAL
        assert "sbt_top_k_dev" in lib.sbt_last_error().decode()
    assert lib.sbt_top_k_dev(None, 10, 2, fake, fake, None) == _lib.SBT_EINVAL
