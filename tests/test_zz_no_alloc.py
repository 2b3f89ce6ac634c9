"""sbt_solve_dev_noalloc (scratch in the library's fixed per-device array,
no allocation) against sbt_solve_dev (caller workspace) through the C ABI:
the same kernels on the same inputs, so every output must be bit-identical.
Two calls in a row, the second on a smaller QUBO with fewer agents, so the
array is reused with the first call's contents still in it; an oversized
request is refused before any device call."""
import numpy as np
import pytest

import trackgen as tg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2402_14718_amd as sbt  # noqa: E402
from paper_2402_14718_amd import _lib  # noqa: E402

KEYS = ("T", "agent_energy", "energy", "best_agent", "c0", "ising_offset", "x", "y", "trace",
        "agent_trace")


def _pair(q, mode, **kw):
    p = sbt.solve_params(**kw)
    a = sbt.DeviceSolver(q, mode, p, want_state=True, want_trace=kw.get("energy_every", 0) > 0)
    b = sbt.DeviceSolver(q, mode, p, want_state=True, want_trace=kw.get("energy_every", 0) > 0)
    a.run()
    ra = a.result()
    b.run_noalloc()
    rb = b.result()
    for k in KEYS:
        va, vb = ra[k], rb[k]
        if va is None:
            assert vb is None, k
        else:
            assert np.array_equal(np.asarray(va), np.asarray(vb)), k
    return ra


def test_noalloc_equals_workspace_solve_twice_second_smaller():
    big = sbt.build_qubo(tg.generate(tg.plain_spec(), 100).hits_struct())
    small = sbt.build_qubo(tg.generate(tg.plain_spec(60), 2).hits_struct())
    assert small.n < big.n
    for mode in ("bsb", "dsb"):
        r1 = _pair(big, mode, agents=256, steps=400, seed=3, energy_every=50)
        r2 = _pair(small, mode, agents=40, steps=300, seed=5, energy_every=30)
        assert r1["x"].shape == (big.n, 256) and r2["x"].shape == (small.n, 40)
    # the streaming kernel and the matrix-core step through the same array
    _pair(small, "dsb", agents=96, steps=200, seed=7, kernel="stream")
    _pair(small, "dsb", agents=96, steps=200, seed=7, kernel="stream_mfma", precision="fp8",
          energy_every=50)


def test_noalloc_refuses_shapes_beyond_its_array():
    q = sbt.build_qubo(tg.generate(tg.plain_spec(), 100).hits_struct())
    p = sbt.solve_params(agents=8192, steps=100)
    need = sbt.workspace_bytes(q.n, q.nnz, "bsb", p)
    assert need > 64 << 20
    ds = sbt.DeviceSolver(q, "bsb", p)          # outputs sized for the request
    with pytest.raises(sbt.SbtError) as e:
        ds.run_noalloc()
    assert e.value.code == _lib.SBT_EINVAL and "limit" in str(e.value)
