"""Plain, slow, float64 CPU oracle for the open-boundary RPY mobility path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP path: the two are fed the
same inputs from ``workloads`` and nothing else.

What it computes (paper section in brackets):

* ``mobility``  - the grand mobility M of eq. (block_mobility) for the
  open-boundary N-body solver [Sec. 3.5, "RPY kernels (NBody)"]: dense
  assembly of the 3N x 3N / 6N x 6N matrix and its product with [F; T]
  [Sec. 3.2, Mdot]; block rows for a subset of particles.
* ``pairloop``  - the same product as a plain C/OpenMP float64 pair loop for
  large N (compiled from ``pairloop.c``).
* ``lanczos``   - M^{1/2} W by the Lanczos iteration the paper uses for
  solvers that only apply M [Sec. 3.3], and the exact symmetric root from an
  eigendecomposition.
* ``gradient``  - the adjoint of U = M(X)[F; T] with respect to X, F and T
  (an addition beside the paper's method, pinned by complex-step
  differentiation of ``mobility``).
* ``drift``     - thermal drift: zero in open space [Sec. 2, Sec. 3.4], and
  the deterministic and random finite-difference divergences of Sec. 4.
* ``integrators`` - the Euler-Maruyama velocities and the stochastic
  Adams-Bashforth step of eq. (bdhi) [Sec. 3.2, Sec. 5.1].
* ``krylov``    - conjugate gradients on M (a Krylov consumer of the product,
  an addition beside the paper's method), pinned against a direct solve and
  CG's finite-termination property.
"""
