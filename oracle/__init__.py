"""CPU FP64 oracle for the particle-interpolation hot path (TEST INFRASTRUCTURE).

This package is the slow, obviously correct reference that the GPU library is
checked against.  It is test infrastructure only: the tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the library itself never does,
and nothing here imports the library.  The two share no code.

What it implements, with the paper passage each part follows (Lalescu, Bramas,
Rampp, Wilczek, "An Efficient Particle Tracking Algorithm for Large-Scale
Parallel Pseudo-Spectral Simulations of Turbulence"):

* ``kernels``   -- the 1-D interpolation polynomials beta_j (Sec. 2.2, the
  tensor-product sum, Eq. "triple_sum"; Lagrange kernels used "for testing
  purposes", spline kernels of smoothness m) and their derivative kernels.
* ``geometry``  -- steps 1-3 of the interpolation algorithm (Sec. 2.2: periodic
  wrap, grid cell, in-cell offset), the bin key and the slice-ordered
  particle grouping with its ``offset`` array (Sec. 3.3.1, "Ordering the
  particles locally").
* ``interp``    -- step 4, the weighted triple sum (Eq. "triple_sum"), and the
  velocity gradient through derivative kernels.
* ``stepping``  -- the tracer ODE dX/dt = u(X) (Eq. "tracers") advanced with
  Euler, Heun and the two-step Adams-Bashforth scheme with its rhs history
  (Sec. 2.2 and Sec. 3.3.1, the *state* and *rhs* arrays).
* ``precision`` -- reduced-precision field storage (per-component scale,
  round-to-nearest-even to BF16 / FP16) emulated bit for bit.
* ``mlp``       -- the learned-correction network's reference forward/backward.
* ``csum.c``    -- the same triple sum as plain C with OpenMP over particles, used
  to time the oracle on host cores and as a third cross-check.

Where the paper is silent the oracle takes one documented reading; each module
states the readings it takes.
"""
