"""Plain FP64 CPU reference of the 3D central-moment lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package exists to prove the GPU path right; the
product (the HIP library and its Python binding) never imports, links or calls
it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may use it.

Everything here follows Premnath & Banerjee, "On the Three-dimensional Central
Moment Lattice Boltzmann Method" (arXiv:1202.6081).  Citations name the
section, equation label or appendix of that paper.

Modules
-------
lattice    velocity sets, orthogonal bases K, monomial/central-moment tables
collision  the per-node collision as its plain definition (central moments of
           f + S relaxed toward the factorized attractors, then mapped back)
lbm        whole-lattice step (push streaming, periodic, half-way bounce-back),
           initial condition, macroscopic fields, totals, kinetic energy

Parity status (the ``-m "not gpu"`` tests):
* the printed tables of the paper (basis matrices, kernel moments, source rows);
* the printed collision cascade, equal to ``collision.collide`` exactly in
  rational arithmetic once its misprints are corrected;
* the D3Q15 source projections m^s of Appendix G, every row, against the K_b
  projections of the continuous raw source moments (binomial theorem on the
  central source moments of Eq. forcingaliased);
* conservation, Galilean invariance, the equilibrium fixed point, and
  closed-form channel and duct flows.
Two choices that no printed value arbitrates are pinned by their own exact
properties only: the density normalisation of the factorized attractors
(``per_mass``), and the D3Q15 source beyond its printed projections.
"""
