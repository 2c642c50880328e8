"""Plain FP64 CPU oracle for the FIT leapfrog hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call anything in this package.
The product path (the HIP library and its Python binding) never imports it
and shares no code with it.

What it computes, in the paper's notation (Sec. II, "Space and Time
Discretization of Maxwell's equations"):

* ``topology``  -- the staggered grid pair and the explicit sparse incidence
  matrices: primal gradient G, primal curl C, primal divergence S, dual curl
  C~ and dual divergence S~, each assembled from its own oriented-incidence
  construction (eqs. maxwell_grid1/2), plus the PEC restriction.
* ``materials`` -- the diagonal material matrices M_eps, M_sigma, M_mu
  (eq. maxwell_grid3) from per-cell values on a uniform or tensor-product
  grid (per-axis cell widths).
* ``leapfrog``  -- the leapfrog update of Sec. II-A with loss and source,
  and the discrete energies of eq. (energy).
* ``stability`` -- the CFL estimate (eq. cfl), the skew matrix A of
  eq. FIT_ode_2 and its spectral norm.
* ``gram``      -- the bilinear energy form <x^(m), x^(n)>_M for a set of
  snapshots.
* ``adjoint``   -- the discrete reverse-time adjoint of the leapfrog
  recurrence and the per-cell gradient of a probe-energy objective.
* ``expm``      -- the action of exp(tA) by scaling and a truncated Taylor
  recurrence (Sec. III-A), with the parameter choice of its docstring, and
  the tolerance of eq. tolerance_leja_2.
* ``leja``      -- the action of exp(tA) by Leja interpolation at conjugate
  pairs of points on the imaginary axis (Sec. III-A).
* ``paraexp``   -- ParaExp (Sec. III, Alg. 1) with leapfrog particular
  solutions and the staggered reconstruction of Sec. III-B.

Every function is FP64 and unblocked.  Pins (tests that tie the oracle to
the paper and to the mathematics) live in ``tests/test_oracle_*.py``.
Functions without such a pin say "parity unpinned" in their docstring;
at present none does.
"""
from . import topology, materials, leapfrog, stability, gram, adjoint, layout, expm, leja, paraexp  # noqa: F401
