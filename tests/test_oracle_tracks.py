"""Pins of the oracle's post-processing and efficiency / purity (Eq. 18-19)."""
import numpy as np

import trackgen as tg
from oracle import qubo, tracks


def test_chain_and_conflict_resolution_by_hand():
    # two tracks 0-1-2-3-4 and 10-11-12-13, plus a branch 2->7 that conflicts
    trip = np.array([[0, 1, 2], [1, 2, 3], [2, 3, 4], [1, 2, 7],
                     [10, 11, 12], [11, 12, 13]])
    T = np.array([1, 1, 1, 1, 1, 1])
    d = tracks.selected_doublets(trip, T)
    assert (2, 7) in d and (2, 3) in d
    res = tracks.resolve_conflicts(d)
    assert (2, 7) not in res and (2, 3) not in res      # hit 2 has two outgoing
    paths = tracks.chain(res)
    assert sorted(paths) == [[0, 1, 2], [3, 4], [10, 11, 12, 13]]
    cands = tracks.track_candidates(trip, T, 4)
    assert cands == [[10, 11, 12, 13]]
    # dropping the branch restores the first track
    T2 = np.array([1, 1, 1, 0, 1, 1])
    assert sorted(tracks.track_candidates(trip, T2, 4)) == [[0, 1, 2, 3, 4], [10, 11, 12, 13]]


def test_score_counts():
    particle = np.array([0, 0, 0, 0, 1, 1, 1, 1, -1])
    layer = np.array([0, 1, 2, 3, 0, 1, 2, 3, 2])
    # particle 0 fully found, particle 1 found with a fake hit 8 in place of 6
    cands = [[0, 1, 2, 3], [4, 5, 8, 7]]
    eff, pur, tp, fn, fp = tracks.score(cands, particle, layer)
    assert (tp, fn, fp) == (4, 2, 2)
    assert eff == 4 / 6 and pur == 4 / 6


def test_true_solution_is_perfect_on_noise_free_event():
    spec = tg.EventSpec(n_particles=15, pt_min=1.0, pt_max=10.0, eta_max=1.0,
                        noise_frac=0.0, radii=tg.RADII_10, sigma_rphi=0.0)
    ev = tg.generate(spec, 31)
    q = qubo.build_event(ev)
    T = tracks.true_triplet_mask(ev, q.trip_hits)
    eff, pur, tp, fn, fp = tracks.evaluate(ev, q.trip_hits, T)
    assert pur == 1.0 and fp == 0
    # every true doublet of a particle with a full 10-hit track is reconstructed
    full = set(p for p in range(15) if np.sum(ev.particle == p) == 10)
    eff_full, pur_full, *_ = tracks.score(
        tracks.track_candidates(q.trip_hits, T, 4), ev.particle, ev.layer, full)
    assert eff_full == 1.0
