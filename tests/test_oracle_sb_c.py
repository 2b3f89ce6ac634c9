"""The C oracle (oracle/sb_omp.c, agents on host threads) against the Python
oracle, bit for bit: same FP64 operations in the same order, so every
position and momentum must be equal, for every mode and thread count.  The
Python oracle itself is pinned by tests/test_oracle_sb.py."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import trackgen as tg
from oracle import ising as oising
from oracle import qubo as oqubo
from oracle import sb as osb
from oracle import sb_c


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(sb_c.LIB):
        sb_c.build()


def _event(spec, seed):
    o = oqubo.build_event(tg.generate(spec, seed))
    return oising.from_qubo(o.a, o.b)


@pytest.mark.parametrize("mode,dt,K", [("bsb", 1.0, 40), ("dsb", 1.0, 40), ("asb", 0.1, 30),
                                       ("bsb", 0.1, 25)])
def test_c_oracle_bit_identical_to_python_oracle(mode, dt, K):
    isg = _event(tg.plain_spec(60), 3)
    ref = osb.run(isg.J, isg.h, isg.c0, mode, 12, K, dt=dt, seed=5, event=2)
    for threads in (1, 3):
        x, y, used = sb_c.run(isg.J, isg.h, isg.c0, mode, 12, K, dt=dt, seed=5, event=2,
                              threads=threads)
        assert used == threads
        assert np.array_equal(x, ref.x) and np.array_equal(y, ref.y), (mode, threads)


def test_c_oracle_random_qubo_and_given_start():
    rng = np.random.default_rng(2)
    n = 50
    A = sp.random(n, n, density=0.1, random_state=3, format="csr")
    b = ((A + A.T) * -1.0).tocsr()
    b.setdiag(0.0)
    b.eliminate_zeros()
    b.sort_indices()
    isg = oising.from_qubo(rng.uniform(0, 1, n), b)
    x0 = rng.uniform(-0.5, 0.5, (n, 7))
    y0 = rng.uniform(-0.5, 0.5, (n, 7))
    for mode in ("bsb", "dsb", "asb"):
        ref = osb.run(isg.J, isg.h, 0.3, mode, 7, 33, dt=0.2, a0=1.5, x0=x0, y0=y0)
        x, y, _ = sb_c.run(isg.J, isg.h, 0.3, mode, 7, 33, dt=0.2, a0=1.5, x0=x0, y0=y0,
                           threads=2)
        assert np.array_equal(x, ref.x) and np.array_equal(y, ref.y), mode


def test_c_oracle_rejects_bad_arguments():
    isg = _event(tg.tiny_spec(), 1)
    with pytest.raises(KeyError):
        sb_c.run(isg.J, isg.h, isg.c0, "xsb", 2, 3)
