"""CPU FP64 oracle for matrix-based omnidirectional pressure integration
(Zigunov & Charonko, "A fast, matrix-based method to perform omnidirectional
pressure integration", arXiv 2311.16935).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the HIP library is checked against.  Only the test-suite, the
smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import it.  The library never calls it, shares no code with it, and the
oracle never imports the library.

Modules
-------
constants  ray-count constants c_jk, A_tot and per-face totals
           (Section "Weight Computation for Arbitrary Boundary Shapes").
counters   per-cell ray counters A_j^i for an arbitrary mask
           (Eqs. Acn, AEnp1, AEn, ANnp1, ANn and their 3-D analogues).
system     explicit sparse assembly of [W^{n+1}], [W^n] and {S}
           (Eqs. ExplicitEqn_FaceCrossing, weights, wcnp1, MatrixEquation).
solve      Algorithm 1 with an exact sparse-LU inner solve (route O1), the
           direct solve of its fixed point (route O2), the residuals of Eqs.
           ResidualPressure / ResidualMomentum, and the per-component gauge.
rays       brute-force ray tracing: counters from explicit rays (face-crossing
           and cell-centred paths), and a rotating-parallel-ray
           omnidirectional integrator on tiny grids.
cellcentered  the 2-D cell-centred scheme: counters by tracing the
           nearest-centre paths over all angles and offsets, and its system.
flow       the velocity -> source stage (Navier-Stokes, RANS, compressible).
unet       FP64 reference of the warm-start network's layers (forward and
           backward), written as plain direct convolutions.

Parity status: every function here is pinned by tests in
``tests/test_oracle_*.py`` against values the paper prints, closed forms,
independent geometric derivations or brute force; none is "parity unpinned".
"""
