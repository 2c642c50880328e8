"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module draws random numbers and paints per-cell material maps; it holds
none of the method's arithmetic (no curl, no averaging, no time stepping).
Both sides receive its arrays as plain data and derive everything else
(edge/facet masks, material matrices, source edge, probe edges) themselves.

Conventions shared by both sides (they name data, they compute nothing):

* A grid has ``nx, ny, nz`` primal CELLS per axis; node (i, j, k) has
  0 <= i <= nx etc.  Per-cell arrays have shape ``(nz, ny, nx)`` (x fastest).
* A per-facet random potential has shape ``(3, nz, ny, nx)``: entry
  ``[a, k, j, i]`` belongs to the facet normal to axis ``a`` anchored at node
  ``(i, j, k)``.  Every interior facet (0 < p_a < n_a) has a slot; slots of
  boundary facets are present but carry values that both sides discard.
* A source is named by (axis, node i, j, k) of one primal edge plus the
  Gaussian waveform parameters (peak current, time width).
* A probe box is a closed node-coordinate box ``[lo, hi]`` per axis.
"""
from .configs import (  # noqa: F401
    WorkloadSpec, dielectric_blocks, lossy_slab, facet_potential,
    centre_source, random_source, batch_sizes, probe_box, c1, c2, c3, c4, c5,
    c2_small, c4_small, c5_small, scaled, EPS0_SI, MU0_SI, x1, x1_graded, steps_for, c3_graded,
)
