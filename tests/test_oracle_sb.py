"""Pins of the oracle's Ising map, SB integrator, energy and brute force."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import trackgen as tg
from oracle import brute, energy, ising, qubo, sb, tracks


def _qubo_csr(n, seed, density=0.3):
    a, b = tg.random_qubo(n, seed, density=density)
    return a, sp.csr_matrix(b), b


# ------------------------------------------------------------- Ising map

def test_qubo_ising_identity_random_T():
    ev = tg.generate(tg.plain_spec(60), 4)
    q = qubo.build_event(ev)
    isg = ising.from_qubo(q.a, q.b)
    rng = np.random.default_rng(0)
    T = (rng.random((q.n, 16)) < 0.5).astype(np.int8)
    s = 2.0 * T - 1.0
    O = energy.qubo_energy(q.a, q.b, T)
    E = ising.ising_energy(isg, s)
    assert np.allclose(O, E + isg.C, rtol=1e-12, atol=1e-12 * np.abs(O).max())


def test_c0_is_population_std_of_all_entries():
    a, bcsr, bdense = _qubo_csr(15, 3)
    isg = ising.from_qubo(a, bcsr)
    Jd = -bdense / 4.0
    assert isg.c0 == pytest.approx(0.5 / (math.sqrt(15) * np.std(Jd)), rel=1e-12)
    assert np.array_equal(isg.J.toarray(), Jd)
    assert np.allclose(isg.h, -(a / 2 + bdense.sum(axis=1) / 4), rtol=0, atol=1e-15)


def test_c0_without_couplings():
    isg = ising.from_qubo(np.array([0.1, 0.2, 0.3, 0.4]), sp.csr_matrix((4, 4)))
    assert isg.c0 == 0.25


# ------------------------------------------------------ energy and brute

def test_energy_matches_quadratic_form():
    a, bcsr, bdense = _qubo_csr(18, 5)
    rng = np.random.default_rng(1)
    T = (rng.random((18, 40)) < 0.5).astype(np.int8)
    O = energy.qubo_energy(a, bcsr, T)
    Tf = T.astype(float)
    expect = Tf.T @ a + np.array([sum(bdense[i, j] * Tf[i, k] * Tf[j, k]
                                      for i in range(18) for j in range(i))
                                  for k in range(40)])
    assert np.allclose(O, expect, rtol=0, atol=1e-12)


def test_brute_force_against_plain_loop():
    a, _, bdense = _qubo_csr(8, 6)
    best = math.inf
    for code in range(256):
        T = [(code >> i) & 1 for i in range(8)]
        o = sum(a[i] * T[i] for i in range(8))
        o += sum(bdense[i, j] * T[i] * T[j] for i in range(8) for j in range(i))
        best = min(best, o)
    e, winners = brute.ground_states(a, bdense)
    assert e == pytest.approx(best, abs=1e-12)
    for w in winners:
        assert energy.qubo_energy(a, sp.csr_matrix(bdense), w) == pytest.approx(best, abs=1e-12)


def test_best_agent_ties_lowest_index():
    assert energy.best_agent(np.array([3.0, -1.0, 2.0, -1.0])) == 1


# -------------------------------------------------------- SB integrator

def _closed_form_free(x0, y0, steps, dt, a0):
    """J = 0, h = 0: each spin follows (x, y) <- M_k (x, y) with
    M_k = [[1 - dt^2 a0 (a0 - a_k), dt a0], [-dt (a0 - a_k), 1]]."""
    v = np.array([x0, y0], dtype=np.float64)
    for k in range(steps):
        g = a0 - a0 * k / steps
        M = np.array([[1.0 - dt * dt * a0 * g, dt * a0], [-dt * g, 1.0]])
        v = M @ v
    return v


@pytest.mark.parametrize("mode", ["bsb", "dsb"])
def test_free_oscillator_matches_matrix_product(mode):
    n, m, K = 6, 3, 40
    J = sp.csr_matrix((n, n))
    h = np.zeros(n)
    r = sb.run(J, h, 0.7, mode, m, K, dt=0.5, a0=1.3, seed=9)
    from oracle.philox import initial_state
    x0, y0 = initial_state(n, m, 9)
    for i in range(n):
        for k in range(m):
            v = _closed_form_free(x0[i, k], y0[i, k], K, 0.5, 1.3)
            assert np.all(np.abs(v) < 1.0)       # no wall in this window
            assert r.x[i, k] == pytest.approx(v[0], rel=1e-13, abs=1e-15)
            assert r.y[i, k] == pytest.approx(v[1], rel=1e-13, abs=1e-15)


def test_wall_is_strict_and_inelastic():
    """One spin, J = 0, h = 1, c0 = 1, a0 = dt = 1, from rest at x = y = 0.
    With K = 1 (a_0 = 0): y = 1, x = 1, which is on the wall but not past it,
    so nothing is clamped.  With K = 2 (a = 0, 1/2): step 0 as before, then
    y = 1 + (1 - 1/2) = 1.5, x = 2.5 -> clamped to (1, 0)."""
    J = sp.csr_matrix((1, 1))
    z = np.zeros((1, 1))
    r = sb.run(J, np.array([1.0]), 1.0, "bsb", 1, 1, x0=z, y0=z)
    assert (r.x[0, 0], r.y[0, 0]) == (1.0, 1.0)
    r = sb.run(J, np.array([1.0]), 1.0, "bsb", 1, 2, x0=z, y0=z)
    assert (r.x[0, 0], r.y[0, 0]) == (1.0, 0.0)
    r = sb.run(J, np.array([-1.0]), 1.0, "dsb", 1, 2, x0=z, y0=z)
    assert (r.x[0, 0], r.y[0, 0]) == (-1.0, 0.0)


def test_coupled_pair_dsb_vs_bsb_by_hand():
    """Two spins, J_01 = 1, h = 0, c0 = 1, a0 = dt = 1, one step (a_0 = 0):
    bSB: y' = y + (x_other - x), x' = x + y';  dSB: y' = y + (sgn(x_other) - x)."""
    J = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
    x0 = np.array([[0.1], [-0.05]])
    y0 = np.array([[0.02], [0.03]])
    rb = sb.run(J, np.zeros(2), 1.0, "bsb", 1, 1, x0=x0, y0=y0)
    rd = sb.run(J, np.zeros(2), 1.0, "dsb", 1, 1, x0=x0, y0=y0)
    yb = [0.02 + (-0.05 - 0.1), 0.03 + (0.1 + 0.05)]
    yd = [0.02 + (-1.0 - 0.1), 0.03 + (1.0 + 0.05)]
    assert np.allclose(rb.y[:, 0], yb, rtol=0, atol=1e-16)
    assert np.allclose(rb.x[:, 0], [0.1 + yb[0], -0.05 + yb[1]], rtol=0, atol=1e-16)
    # dSB: x0 + y' = 0.1 - 1.08 = -0.98 (inside), -0.05 + 1.08 = 1.03 (wall)
    assert np.allclose(rd.x[:, 0], [0.1 + yd[0], 1.0], rtol=0, atol=1e-16)
    assert np.allclose(rd.y[:, 0], [yd[0], 0.0], rtol=0, atol=1e-16)


@pytest.mark.parametrize("mode", ["bsb", "dsb"])
def test_sign_symmetry_without_field(mode):
    ev = tg.generate(tg.plain_spec(40), 8)
    q = qubo.build_event(ev)
    isg = ising.from_qubo(q.a, q.b)
    from oracle.philox import initial_state
    x0, y0 = initial_state(q.n, 4, 17)
    assert np.all(x0 != 0)
    h0 = np.zeros(q.n)
    r1 = sb.run(isg.J, h0, isg.c0, mode, 4, 200, x0=x0, y0=y0)
    r2 = sb.run(isg.J, h0, isg.c0, mode, 4, 200, x0=-x0, y0=-y0)
    assert np.array_equal(r1.x, -r2.x) and np.array_equal(r1.y, -r2.y)


def test_agents_are_independent_shots():
    ev = tg.generate(tg.plain_spec(30), 9)
    q = qubo.build_event(ev)
    isg = ising.from_qubo(q.a, q.b)
    r_all = sb.run(isg.J, isg.h, isg.c0, "dsb", 6, 100, seed=3)
    from oracle.philox import initial_state
    x0, y0 = initial_state(q.n, 6, 3)
    r_one = sb.run(isg.J, isg.h, isg.c0, "dsb", 1, 100, x0=x0[:, 4:5], y0=y0[:, 4:5])
    assert np.array_equal(r_all.x[:, 4:5], r_one.x)


@pytest.mark.parametrize("mode", ["bsb", "dsb"])
def test_sb_reaches_brute_force_ground_state(mode):
    """Heuristic: 32 agents x 2000 steps find the exact minimum of most
    small random QUBOs with track-like sparsity (about two couplings per
    variable); the rate is asserted at 90%."""
    hits = 0
    total = 0
    for seed in range(40):
        a, bcsr, bdense = _qubo_csr(14, 100 + seed, density=0.15)
        e_min, _ = brute.ground_states(a, bdense)
        isg = ising.from_qubo(a, bcsr)
        r = sb.run(isg.J, isg.h, isg.c0, mode, 32, 2000, seed=seed)
        E = energy.qubo_energy(a, bcsr, sb.readout(r.x))
        total += 1
        hits += int(E.min() <= e_min + 1e-9)
        assert E.min() >= e_min - 1e-9
    assert hits >= 0.9 * total


def test_true_tracks_are_single_flip_local_minimum():
    """Noise-free 4-layer events: switching a true triplet off loses its
    quadruplet reward (S <= 1 outweighs a_i), switching a fake on adds a
    conflict (+1) that no reward S <= 1 pays back."""
    for seed in range(1, 6):
        ev = tg.generate(tg.tiny_spec(), seed)
        q = qubo.build_event(ev)
        T = tracks.true_triplet_mask(ev, q.trip_hits)
        e0 = energy.qubo_energy(q.a, q.b, T)
        for i in range(q.n):
            T2 = T.copy()
            T2[i] ^= 1
            assert energy.qubo_energy(q.a, q.b, T2) > e0


def test_tiny_event_solution_reconstructs_every_track():
    ev = tg.generate(tg.tiny_spec(), 2)
    q = qubo.build_event(ev)
    isg = ising.from_qubo(q.a, q.b)
    r = sb.run(isg.J, isg.h, isg.c0, "dsb", 32, 2000, seed=1)
    E = energy.qubo_energy(q.a, q.b, sb.readout(r.x))
    best = energy.best_agent(E)
    T = sb.readout(r.x)[:, best]
    assert np.array_equal(T, tracks.true_triplet_mask(ev, q.trip_hits))
    eff, pur, *_ = tracks.evaluate(ev, q.trip_hits, T)
    assert eff == 1.0 and pur == 1.0


def test_asb_single_oscillator_converges_to_the_ode():
    """aSB with J = 0, h = 0 is dx/dt = a0 y, dy/dt = -(x^2 + a0 - a(t)) x
    (Eq. 1-2) with a(t) = a0 t / T.  Symplectic Euler converges to the exact
    trajectory at first order in dt: halving dt halves the error."""
    from scipy.integrate import solve_ivp
    a0, T = 1.0, 3.0
    x0, y0 = np.array([[0.3]]), np.array([[-0.2]])

    def rhs(t, u):
        return [a0 * u[1], -(u[0] ** 2 + a0 - a0 * t / T) * u[0]]

    exact = solve_ivp(rhs, (0.0, T), [0.3, -0.2], rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for K in (3000, 6000):
        r = sb.run(sp.csr_matrix((1, 1)), np.zeros(1), 0.5, "asb", 1, K, dt=T / K, a0=a0,
                   x0=x0, y0=y0)
        errs.append(abs(r.x[0, 0] - exact[0]) + abs(r.y[0, 0] - exact[1]))
    assert errs[0] < 3e-3
    assert 1.6 < errs[0] / errs[1] < 2.4


def test_asb_has_no_walls_and_odd_symmetry():
    rng = np.random.default_rng(3)
    n = 12
    A = sp.random(n, n, density=0.4, random_state=5, data_rvs=lambda k: rng.normal(0, 1, k))
    J = sp.csr_matrix(A + A.T)
    x0 = rng.uniform(-0.1, 0.1, (n, 4))
    y0 = rng.uniform(-0.1, 0.1, (n, 4))
    # (explicit steps of the cubic force need a small dt: at c0 = 2, dt = 0.2
    # this system diverges)
    r1 = sb.run(J, np.zeros(n), 1.0, "asb", 4, 200, dt=0.1, x0=x0, y0=y0)
    r2 = sb.run(J, np.zeros(n), 1.0, "asb", 4, 200, dt=0.1, x0=-x0, y0=-y0)
    assert np.all(np.isfinite(r1.x))
    assert np.array_equal(r1.x, -r2.x) and np.array_equal(r1.y, -r2.y)
    # the coupling carries positions past 1, which bSB's wall forbids
    assert np.abs(r1.x).max() > 1.0
    rb = sb.run(J, np.zeros(n), 1.0, "bsb", 4, 200, dt=0.1, x0=x0, y0=y0)
    assert np.abs(rb.x).max() <= 1.0


# ------------------------------------------------ checkpoints and margins

def _dense_objective(a, bdense, T):
    """Eq. 13 as a dense quadratic form per column of T (j < i pairs)."""
    T = np.asarray(T, dtype=np.float64)
    return T.T @ a + np.einsum("ik,ij,jk->k", T, np.tril(bdense, -1), T)


@pytest.mark.parametrize("every", [1, 3, 4, 7])
def test_checkpoint_energies_follow_the_free_oscillator(every):
    """J = 0, h = 0: every spin follows the 2x2 matrix product, so the
    readout after step k is known independently; the checkpoint energies of
    an unrelated QUBO (a, b) are then its dense quadratic form at those T,
    recorded after steps every, 2 every, ... (odd `every` puts checkpoints
    on odd steps), and the trace is their running minimum over agents."""
    n, m, K, dt, a0 = 7, 5, 29, 0.5, 1.3
    a, bcsr, bdense = _qubo_csr(n, 12, density=0.5)
    from oracle.philox import initial_state
    x0, y0 = initial_state(n, m, 4)
    r = sb.run(sp.csr_matrix((n, n)), np.zeros(n), 0.9, "bsb", m, K, dt=dt, a0=a0, seed=4,
               ckpt_every=every, qubo=(a, bcsr))
    n_ck = K // every
    assert r.agent_trace.shape == (n_ck, m) and r.trace.shape == (n_ck,)
    best = math.inf
    for c in range(n_ck):
        k = (c + 1) * every
        T = np.zeros((n, m), dtype=np.int8)
        for i in range(n):
            for j in range(m):
                v = np.array([x0[i, j], y0[i, j]])
                for s in range(k):
                    g = a0 - a0 * s / K
                    v = np.array([[1.0 - dt * dt * a0 * g, dt * a0], [-dt * g, 1.0]]) @ v
                T[i, j] = 1 if v[0] >= 0 else 0
        expect = _dense_objective(a, bdense, T)
        assert np.allclose(r.agent_trace[c], expect, rtol=0, atol=1e-12), c
        best = min(best, float(expect.min()))
        assert r.trace[c] == pytest.approx(best, abs=1e-12)
    assert np.all(np.diff(r.trace) <= 0)


def test_last_checkpoint_is_the_final_readout():
    ev = tg.generate(tg.plain_spec(30), 5)
    q = qubo.build_event(ev)
    isg = ising.from_qubo(q.a, q.b)
    r = sb.run(isg.J, isg.h, isg.c0, "dsb", 6, 60, seed=2, ckpt_every=20, qubo=(q.a, q.b))
    E = energy.qubo_energy(q.a, q.b, sb.readout(r.x))
    assert np.array_equal(r.agent_trace[-1], E)
    assert r.trace[-1] == min(r.agent_trace.min(), E.min())


def test_checkpoints_need_a_qubo():
    with pytest.raises(ValueError):
        sb.run(sp.csr_matrix((2, 2)), np.zeros(2), 1.0, "bsb", 1, 4, ckpt_every=2)


def test_sign_margin_is_the_smallest_position_used_by_hand():
    """dSB, J = 0, h = 0, a0 = 1, dt = 1/2, two steps (a_0 = 0, a_1 = 1/2).
    Spin 0 starts at x = 2^-23, y = 0: step 0 gives y = -2^-24, x =
    2^-23 - 2^-25 = 3 * 2^-25; step 1 gives y = -2^-24 - 3 * 2^-27 and
    x = 3 * 2^-25 - 2^-25 - 3 * 2^-28 = 13 * 2^-28.  Spin 1 stays far
    from zero.  The margin over two steps is the smallest |x| whose sign was
    used (2^-23, 3 * 2^-25) or read out (13 * 2^-28): 13 * 2^-28 ~ 4.8e-8;
    over one step it is still the final readout."""
    x0 = np.array([[2.0 ** -23], [0.5]])
    y0 = np.zeros((2, 1))
    J = sp.csr_matrix((2, 2))
    r = sb.run(J, np.zeros(2), 1.0, "dsb", 1, 2, dt=0.5, x0=x0, y0=y0, margin_steps=2)
    assert r.x[0, 0] == 13 * 2.0 ** -28
    assert r.sign_margin[0] == 13 * 2.0 ** -28
    # a start nearer zero than anything after it is caught at step 0
    x0 = np.array([[-(2.0 ** -30)], [0.5]])
    y0 = np.array([[-(2.0 ** -10)], [0.0]])
    r = sb.run(J, np.zeros(2), 1.0, "dsb", 1, 2, dt=0.5, x0=x0, y0=y0, margin_steps=2)
    assert r.sign_margin[0] == 2.0 ** -30
    # margins are per agent: a second agent far from zero keeps its own
    x0 = np.array([[2.0 ** -23, 0.25], [0.5, -0.5]])
    r = sb.run(J, np.zeros(2), 1.0, "dsb", 2, 2, dt=0.5, x0=x0, y0=np.zeros((2, 2)),
               margin_steps=2)
    assert r.sign_margin[0] == 13 * 2.0 ** -28 and r.sign_margin[1] > 0.1


def test_wall_margin_is_the_closest_approach_to_the_wall_by_hand():
    """bSB, J = 0, h = 0, a0 = dt = 1, one step (a_0 = 0): y' = y - x,
    x' = x + y' = y, exact for dyadic values.  Agent 0 lands at 1 - 2^-20
    (inside, margin 2^-20), agent 1 at 1 + 2^-21 (clamped, margin 2^-21),
    agent 2 at -(1 - 2^-22) (margin 2^-22, sign irrelevant)."""
    x0 = np.array([[0.5, 0.25, -0.5]])
    y0 = np.array([[1.0 - 2.0 ** -20, 1.0 + 2.0 ** -21, -(1.0 - 2.0 ** -22)]])
    r = sb.run(sp.csr_matrix((1, 1)), np.zeros(1), 1.0, "bsb", 3, 1, x0=x0, y0=y0,
               margin_steps=1)
    assert list(r.wall_margin) == [2.0 ** -20, 2.0 ** -21, 2.0 ** -22]
    assert r.x[0, 1] == 1.0 and r.y[0, 1] == 0.0
    # steps past margin_steps are not logged
    r = sb.run(sp.csr_matrix((1, 1)), np.zeros(1), 1.0, "bsb", 3, 1, x0=x0, y0=y0,
               margin_steps=0)
    assert np.all(np.isinf(r.wall_margin))
