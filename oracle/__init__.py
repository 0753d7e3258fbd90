"""Plain FP64 CPU oracle of the third-order gas-kinetic scheme on triangles.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library: it consumes the
same seeded arrays from ``gks_inputs`` and nothing else.

It computes, slowly and literally, what the method defines:

* ``mesh``     cell and face geometry, face Gauss points (section 2.1,
               Eq. fluxgauss; section 3.1, Eqs. RCP and h)
* ``cls``      the compact least-squares conditions and their least-squares
               solution by a direct sparse solve (section 3.1, Eqs.
               spdConserved, A:B:b, A:B:b:3; section 3.2, Eq. spdConserved:5)
* ``kinetic``  Maxwellian moments, slope inversion, the time coefficients and
               the third-order BGK flux at one Gauss point (section 2.2, Eqs.
               generalSolution, fNS, 3orderf0:2, Nomenclature1-2, 3orderg:2;
               section 4, Eqs. tauIns and tauVis)
* ``scheme``   Gauss-point states, face fluxes, the finite-volume update and
               the time-step rule (section 2.1, Eq. fvm3)

Every function states the passage it follows.  The linear solve uses a
library direct solver: GMRES, reverse Cuthill-McKee and ILU are devices for
reaching the same solution and do not appear here.
"""
