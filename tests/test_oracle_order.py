"""Pins of the oracle's spin relabelling: the azimuth key against the
library atan2, the order on hand-placed hits, and the invariance of the
objective (Eq. 13) under relabelling."""
import numpy as np
import scipy.sparse as sp

import trackgen as tg
from oracle import energy as oenergy
from oracle import order as oorder
from oracle import qubo as oqubo


def test_key_is_monotone_in_the_azimuth():
    rng = np.random.default_rng(5)
    r = rng.uniform(1, 1000, 50000)
    phi = rng.uniform(0, 2 * np.pi, 50000)
    x, y = r * np.cos(phi), r * np.sin(phi)
    ang = np.mod(np.arctan2(y, x), 2 * np.pi)
    key = oorder.diamond_key(x, y)
    o = np.argsort(ang)
    assert np.all(np.diff(key[o]) >= 0)
    assert np.all((key >= 0) & (key < 4))


def test_key_at_the_axes():
    assert oorder.diamond_key([5.0, 0.0, -2.0, 0.0, 0.0], [0.0, 3.0, 0.0, -7.0, 0.0]).tolist() \
        == [0.0, 1.0, 2.0, 3.0, 0.0]
    # just below the positive x axis the key approaches 4
    assert oorder.diamond_key(1.0, -1e-9) > 3.999


def test_order_on_hand_placed_hits():
    # five triplets whose middle hits sit at 100, 10, 350, 190 and 10 degrees
    # (the last two at 10 degrees differ in z)
    deg = np.array([100.0, 10.0, 350.0, 190.0, 10.0])
    z = np.array([0.0, 5.0, 0.0, 0.0, -5.0])
    ids = np.arange(100, 105)
    x, y = 50 * np.cos(np.radians(deg)), 50 * np.sin(np.radians(deg))
    trip = np.stack([ids * 0, ids, ids * 0], axis=1)
    perm = oorder.phi_order(trip, ids, x, y, z)
    assert perm.tolist() == [4, 1, 0, 3, 2]


def test_relabelling_keeps_every_energy():
    ev = tg.generate(tg.plain_spec(80), 4)
    q = oqubo.build_event(ev)
    perm = oorder.phi_order(q.trip_hits, ev.hit_id, ev.x, ev.y, ev.z)
    assert sorted(perm.tolist()) == list(range(q.n))
    a2, b2, th2 = oorder.permute(q.a, q.b, q.trip_hits, perm)
    assert np.array_equal(th2, q.trip_hits[perm])
    assert abs(b2 - b2.T).max() == 0
    rng = np.random.default_rng(1)
    T = (rng.random((q.n, 8)) < 0.3).astype(np.int8)
    e1 = oenergy.qubo_energy(q.a, q.b, T)
    e2 = oenergy.qubo_energy(a2, b2, T[perm])
    assert np.allclose(e1, e2, rtol=1e-13, atol=1e-12)
    # coupled triplets end up closer together
    def spread(b):
        b = sp.coo_matrix(b)
        return np.median(np.abs(b.row - b.col))
    assert spread(b2) < spread(q.b)
