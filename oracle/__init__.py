"""Plain FP64 CPU oracle of the HWENO-GR finite-volume scheme.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP path is checked against.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path (the C-ABI library and its Python binding) never does, and this package
imports nothing from the product path.

Layout of a state (same convention the tests hand to both sides):

* 1D: ``U[m, c, i]`` with ``m`` in {0: cell average, 1: scaled xi-moment},
  ``c`` in {rho, rho*u, E}, ``i`` the cell index.
* 2D: ``U[m, c, j, i]`` with ``m`` in {0: average, 1: xi-moment,
  2: eta-moment}, ``c`` in {rho, rho*u, rho*v, E}, ``j`` the y index and
  ``i`` the x index (x fastest).

Every routine works on float64 arrays and, unchanged, on complex128 arrays:
non-analytic operations (abs, max, min, comparisons) act on the real part
only, so that ``Im(F(U + i*h*dU))/h`` is the exact directional derivative
(complex-step tangent-linear model) along the branch taken at ``Re(U)``.

Modules:

* ``common``  -- quadrature rules, complex-safe helpers, gas physics,
  characteristic bases, the positivity-preserving flux bound.
* ``recon``   -- scalar HWENO reconstruction with unified stencils (1D, 2D),
  built from the moment conditions of the paper's Appendix A.
* ``scheme1d``/``scheme2d`` -- ghost cells, the semi-discrete residual
  (conservative reconstruction, positivity limiter, weak-derivative moments,
  gradient reconstruction, fluxes, assembly).
* ``rk``      -- the SSP-RK3 driver with modified moments, the time-step rule
  and the stage-admissibility restart.
* ``mms``     -- manufactured-solution sources of Examples 5.1 and 5.2.
"""

from .common import Physics, Options  # noqa: F401
