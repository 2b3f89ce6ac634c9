"""The QUBO built on the GPU (sbt_build_qubo_gpu, through the C ABI) against
the FP64 oracle's construction: doublet / triplet / quadruplet enumeration,
triplet order, CSR structure and hit ids bit-exact.  Values: exp (Eq. 15)
and atan2 (Eq. 14) come from the device math library, each within an ulp
of the host's; a = alpha (1 - e^-x) + beta (1 - e^-y) turns an ulp of e^-x
(2^-53 near 1) into an absolute error, so |da| <= 2 (alpha + beta) 2^-52;
b (quadruplet strengths near 1 and +1 conflicts) within two ulps."""
import numpy as np
import pytest

import trackgen as tg
from oracle import qubo as oqubo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2402_14718_amd as sbt  # noqa: E402
from paper_2402_14718_amd import _lib  # noqa: E402


def _ulps_close(x, y, ulps=2):
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    return np.all(np.abs(x - y) <= ulps * np.spacing(np.maximum(np.abs(x), np.abs(y))))


def _same(qg, ref_n, ref_row_ptr, ref_col, ref_b, ref_a, ref_trip):
    assert qg.n == ref_n
    assert np.array_equal(qg.trip_hits, ref_trip)
    assert np.array_equal(qg.row_ptr, ref_row_ptr)
    assert np.array_equal(qg.col, ref_col)
    assert np.all(np.abs(qg.a - ref_a) <= 2 * (0.5 + 0.2) * 2.0 ** -52)
    assert _ulps_close(qg.b, ref_b)


def _oracle_params(p):
    return oqubo.BuildParams(z0_max=p.z0_max, min_track_hits=p.min_track_hits,
                             dphi_tan=p.dphi_tan)


@pytest.mark.parametrize("spec,seed", [
    (tg.tiny_spec(), 1), (tg.tiny_spec(), 4), (tg.plain_spec(), 100), (tg.plain_spec(), 104),
    (tg.plain_spec(300), 9), (tg.EventSpec(n_particles=300, eta_max=0.6, noise_frac=0.3), 9),
    (tg.precision_spec(), 200)])
def test_gpu_build_matches_oracle(spec, seed):
    ev = tg.generate(spec, seed)
    qg, t = sbt.build_qubo_gpu(ev.hits_struct())
    o = oqubo.build_event(ev)
    _same(qg, o.n, o.b.indptr, o.b.indices, o.b.data, o.a, o.trip_hits)
    assert t > 0.0


@pytest.mark.parametrize("variant", ["z0", "four_hits", "wide_window"])
def test_gpu_build_parameter_variants(variant):
    ev = tg.generate(tg.plain_spec(120) if variant != "wide_window" else tg.tiny_spec(), 5)
    p = sbt.build_params_default()
    if variant == "z0":
        p.z0_max = 150.0
    elif variant == "four_hits":
        p.min_track_hits = 4          # no five-hit rule
    else:
        p.dphi_tan = 1e9              # window covers every outer hit
    qg, _ = sbt.build_qubo_gpu(ev.hits_struct(), p)
    qh = sbt.build_qubo(ev.hits_struct(), p)
    _same(qg, qh.n, qh.row_ptr, qh.col, qh.b, qh.a, qh.trip_hits)
    if variant != "wide_window":
        o = oqubo.build_event(ev, _oracle_params(p))
        _same(qg, o.n, o.b.indptr, o.b.indices, o.b.data, o.a, o.trip_hits)


def test_gpu_build_stress_event_matches_host_builder():
    """5000 particles with the stress recipe's doublet z0 cut (N ~ 2.1e5):
    against the host builder, which is bit-exact with the oracle."""
    ev = tg.generate(tg.stress_spec(), 300)
    p = sbt.build_params_default()
    p.z0_max = tg.STRESS_Z0_MAX
    qg, t = sbt.build_qubo_gpu(ev.hits_struct(), p)
    qh = sbt.build_qubo(ev.hits_struct(), p)
    assert qg.n > 200000
    _same(qg, qh.n, qh.row_ptr, qh.col, qh.b, qh.a, qh.trip_hits)


def test_gpu_build_edge_cases():
    ev = tg.generate(tg.plain_spec(80), 3)
    hits = ev.hits_struct()
    perm = np.random.default_rng(1).permutation(hits.shape[0])
    q1, _ = sbt.build_qubo_gpu(hits)
    q2, _ = sbt.build_qubo_gpu(hits[perm])        # input order does not matter
    assert np.array_equal(q1.col, q2.col) and np.array_equal(q1.b, q2.b)
    empty, _ = sbt.build_qubo_gpu(hits[:0])
    assert empty.n == 0 and empty.nnz == 0
    dup = hits.copy()
    dup["hit_id"][5] = dup["hit_id"][4]
    with pytest.raises(sbt.SbtError) as e:
        sbt.build_qubo_gpu(dup)
    assert e.value.code == _lib.SBT_EINVAL
    p = sbt.build_params_default()
    p.min_track_hits = 6
    with pytest.raises(sbt.SbtError) as e:
        sbt.build_qubo_gpu(hits, p)
    assert e.value.code == _lib.SBT_EUNSUPPORTED
