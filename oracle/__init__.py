"""CPU reference ("oracle") for the simulated-bifurcation track-QUBO path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python
binding imports, links or calls this package; only the tests, the smoke
check and the CPU-baseline leg of the benchmark do.  It shares no code with
the HIP library: the only thing both sides use is the seeded input
generator package ``trackgen`` (which holds none of the method's
arithmetic).

Everything here is plain FP64 NumPy/SciPy written for readability, each
function citing the passage of the paper (Okawa, Zeng, Tao, Yung,
"Quantum-Annealing-Inspired Algorithms for Track Reconstruction at
High-Energy Colliders") that it follows:

* ``philox``  -- Philox4x32-10 counter-based generator (Salmon et al. 2011),
                 used only for the SB initial state, which the paper leaves
                 unstated.
* ``qubo``    -- doublets, triplets (Eq. 16), quadruplets (Eq. 17), the
                 five-hit rule, bias weights (Eq. 15) and couplings (Eq. 13,
                 Eq. 14): section "QUBO Formulation" and "QUBO Generation and
                 Track Finding".
* ``ising``   -- the QUBO -> Ising map and the coupling scale c0.
* ``sb``      -- bSB (Eq. 5-8) and dSB (Eq. 9-12) integrated by symplectic
                 Euler, section "Simulated Bifurcation".
* ``energy``  -- the QUBO objective O(a, b, T) of Eq. 13 in FP64 and the
                 best-shot selection of the Results section.
* ``brute``   -- exhaustive ground states for tiny QUBOs.
* ``tracks``  -- post-processing into track candidates and efficiency /
                 purity (Eq. 18-19).
"""
