"""CPU oracle of the stochastic conservative field transfer (TEST INFRASTRUCTURE).

A plain, slow, FP64 numpy/scipy implementation of what the GPU path computes,
written from the paper (Paudel, Smith, Merson, "A Stochastic Conservative Field
Transfer Method for Black-box Multiscale and Multiphysics Coupling"), sec. 2
and sec. 4, and from the sampling specification below.  Only the test suite,
the package smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does, and this package imports nothing from the product.

Modules
-------
philox      Philox4x32-10 counter-based generator and (0,1) conversions
sampling    per-element uniform samples: Osada map (triangles), sorted
            spacings (tetrahedra), affine map to physical points
geometry    element measures, P1 mass matrix (closed form and quadrature),
            lumped mass, degree-2 simplex quadrature
source      mesh-backed P1 source: point localization and evaluation
cvmc        the control-variate Monte Carlo transfer, steps 1-7 of sec. 4.1
supermesh   exact intersection-based load vector on small 2D meshes (sec. 3,
            the definition of b the estimator converges to)

Parity status of each function is stated in its docstring; every function is
pinned by a test in ``tests/test_oracle_*.py`` against an independent fact
(library routine, closed form, identity, brute force or statistics).
"""
