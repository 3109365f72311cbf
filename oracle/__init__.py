"""CPU FP64 oracle for the Multiscale Robin Coupled Method (MRCM) Darcy solve.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library and its Python
binding never do, and the two share no code.  Inputs come from the separate
``inputs`` package, which holds data only.

Contents
--------
* ``discretization`` - geometry, face laws (cell-centred TPFA, the
  trapezoidal-quadrature form of lowest-order Raviart-Thomas mixed elements
  on a Cartesian grid), the Robin face law of eq. (mrc1) with the Robin
  parameter of eq. (beta), and the interface spaces of section 3;
* ``fine`` - the global fine-grid solve of eq. (Darcy) (reference for pins);
* ``mrcm`` - the MRCM itself: local Robin problems (mrc1), basis functions,
  the interface system (mrc2), composition, stitch and the conservation
  check; plus the monolithic form used to pin the static condensation;
* ``transport`` - the sequential-implicit transport of section 4: implicit
  Euler with first-order upwind fluxes, Newton's method with the
  inflection-point strategy, and the sequential loop with the Darcy solve;
* ``cnn`` - the FP64 reference of the learned surrogate (not part of the
  paper's method).
"""
