"""CPU FP64 oracle for real-time TDKS propagation of Bloch orbitals with the
two-step Brillouin-zone sampling of Sato, "Two-step Brillouin zone sampling
for efficient computation of electron dynamics in solids" (arXiv:2112.00920).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the graft
entry point and the CPU-baseline leg of the benchmark may import this package.
The HIP library and its Python binding never import, link or call it, and it
never imports them: the two sides share no code, only the seeded inputs of the
``workloads`` package.

Everything here is plain NumPy in float64/complex128, written for reading
against the paper, not for speed:

* ``cell``        geometry, real-space grid, 4th-order finite differences
* ``kpoints``     Monkhorst-Pack grid (Eq. 8), shifted grids (Eq. 10), Halton
* ``pseudo``      Gaussian local potential and s+p Kleinman-Bylander projectors
* ``hamiltonian`` h_k(t) of Eq. (2) applied to orbitals; dense matrix builder
* ``hxc``         Hartree (FFT Poisson) + Slater exchange + PZ81 correlation
* ``propagate``   Taylor-4 step, density (Eq. 3), current (Eqs. 5-6), runs
* ``ground``      SCF ground state by dense diagonalisation
* ``spectra``     induced current -> sigma, epsilon (Eqs. 12-14), HHG (Eq. 16)

Parity status: every function above is pinned by a CPU test against a closed
form, an invariant, a brute-force computation or a textbook routine (see the
``tests/test_oracle_*.py`` files).  The physical Si spectra of the paper's
figures are "parity unpinned": the figures hold no data and the HGH
pseudopotential, PW92 functional and the Octopus code are not available.
"""
