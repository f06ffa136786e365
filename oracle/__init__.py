"""Plain, slow, float64 CPU oracle for the 2-D vortex-particle FMM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import or call this package; only the test-suite, the
smoke check and the benchmark's CPU-baseline leg do.  It shares no code,
tables or constants with the GPU implementation.

It follows Cruz & Barba, "Characterization of the errors of the Fast Multipole
Method approximation in particle simulations" (2008), in the paper's own
notation:

* ``kernel``   -- regularised Biot-Savart kernel (eq. 6), singular far-field
  kernel (eq. 15 / eq. 27), the O(N^2) direct sum (eq. 7 / eq. 9) and the
  near/far "hybrid" brute-force sum that the FMM approximates;
* ``quadtree`` -- root box, levels, parent/child/neighbour, local list and
  interaction list (Section 3.3.1, Fig. 6-8);
* ``fmm``      -- P2M (eq. 20-21), M2M (Section 3.3.2), M2L (eq. 22),
  L2L (Section 3.3.3), L2P, P2P and the upward / downward sweeps (Fig. 3);
* ``bounds``   -- kernel-substitution error estimate (Section 4.1, Table 1)
  and the multipole truncation bound (Section 4.2, eq. 30-31);
* ``metrics``  -- error normalised by the maximum velocity (Section 5.1);
* ``advect``   -- particles moved with their own velocity (eq. 5), Heun's
  two-stage Runge-Kutta method;
* ``mlp``      -- float64 reference of the parameter-selector network.

Every function is pinned by tests under ``tests/`` against closed forms,
invariants, brute force or values printed in the paper.  Readings of garbled or
silent passages are listed in the module that applies them.
"""
