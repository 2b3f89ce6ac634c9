"""Whole solves captured in a HIP graph (through torch.cuda.CUDAGraph) must
replay bit-identically to eager runs, with eager work between replays."""
import numpy as np
import pytest

import trackgen as tg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2402_14718_amd as sbt  # noqa: E402


def _capture(run):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()              # first launch on this stream outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        run()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("mode,kernel", [("dsb", "resident"), ("dsb", "stream"), ("bsb", "stream"),
                                         ("bsb", "stream_tile"), ("dsb", "stream_mfma")])
def test_single_event_solve_replays_bit_identically(mode, kernel):
    """A whole solve captured in a HIP graph, its one-off preparation
    included (bSB streaming: the row-quad lists; tiled: the tile plan;
    matrix cores: the block plan and the conversions to and from the step's
    tiled state, FP32 couplings as three BF16 terms)."""
    ev = tg.generate(tg.plain_spec(), 100)
    q = sbt.build_qubo(ev.hits_struct())
    p = sbt.solve_params(agents=128, steps=2000 if kernel == "resident" else 400, seed=3,
                         kernel=kernel, energy_every=100)
    ds = sbt.DeviceSolver(q, mode, p, want_state=True, want_trace=True)
    ds.run()
    ref = ds.result()
    g = _capture(ds.run)
    for rep in range(3):
        ds.x.zero_()
        ds.agent_energy.fill_(0.0)
        other = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        r = ds.result()
        assert np.array_equal(r["x"], ref["x"]), rep
        assert np.array_equal(r["agent_energy"], ref["agent_energy"])
        assert np.array_equal(r["trace"], ref["trace"])
        assert r["best_agent"] == ref["best_agent"]
        assert float(other) == float(other)


def test_batch_solve_replays_bit_identically():
    qs = [sbt.build_qubo(tg.generate(s, e).hits_struct()) for s, e in tg.batching_specs()[:6]]
    p = sbt.solve_params(agents=64, steps=600, seed=1, energy_every=100)
    ds = sbt.DeviceBatchSolver(qs, "dsb", "fp16", p, want_agent_energy=True, want_trace=True)
    ds.run()
    ref = ds.result()
    g = _capture(ds.run)
    for rep in range(3):
        ds.best_energy.fill_(0.0)
        ds.agent_energy.fill_(0.0)
        torch.randn(1 << 20, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        r = ds.result()
        assert np.array_equal(r["agent_energy"], ref["agent_energy"]), rep
        assert np.array_equal(r["energy"], ref["energy"])
        assert np.array_equal(r["trace"], ref["trace"])
        for e in range(len(qs)):
            assert np.array_equal(r["T"][e], ref["T"][e])
