"""sbt_top_k_dev against a lexicographic (energy, agent) sort in NumPy:
random energies with many ties, NaN entries, k from 1 to all agents,
agent counts around the workgroup size; and the best agent of a solve."""
import numpy as np
import pytest

import paper_2402_14718_amd as sbt
import trackgen as tg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)


def _reference(e, k):
    key = np.where(np.isnan(e), np.inf, e)
    nan = np.isnan(e).astype(np.int8)
    order = np.lexsort((np.arange(e.size), key, nan))  # NaN last, then energy, then agent
    return e[order[:k]], order[:k]


@pytest.mark.parametrize("agents", [1, 37, 512, 1023, 1024, 1025, 5000])
@pytest.mark.parametrize("ties", [False, True])
def test_top_k_matches_lexicographic_sort(agents, ties):
    rng = np.random.default_rng(agents + 7 * ties)
    e = rng.normal(-100.0, 5.0, agents)
    if ties:
        e = np.round(e)  # many equal energies: order by agent
        e[rng.integers(0, agents, max(1, agents // 10))] = np.nan
    d = torch.from_numpy(e).cuda()
    for k in sorted({1, min(5, agents), min(32, agents), agents}):
        v, i = sbt.top_k(d, k)
        ev, ei = _reference(e, k)
        assert np.array_equal(i.cpu().numpy(), ei), (agents, k)
        got = v.cpu().numpy()
        assert np.array_equal(np.isnan(got), np.isnan(ev)) and np.array_equal(got[~np.isnan(got)],
                                                                               ev[~np.isnan(ev)])


def test_top_k_first_is_the_solve_best_agent():
    q = sbt.build_qubo(tg.generate(tg.plain_spec(), 100).hits_struct())
    s = sbt.DeviceSolver(q, "bsb", sbt.solve_params(agents=256, steps=300, seed=2))
    s.run()
    v, i = sbt.top_k(s.agent_energy, 32)
    r = s.result()
    assert int(i[0]) == r["best_agent"] and float(v[0]) == r["energy"]
    ev, ei = _reference(r["agent_energy"], 32)
    assert np.array_equal(i.cpu().numpy(), ei) and np.array_equal(v.cpu().numpy(), ev)
