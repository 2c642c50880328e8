"""MI355X (gfx950) FIT leapfrog: Python binding of libfit.so.

The kernels and the C ABI live in ``csrc/`` and ``include/fit.h``; this
package only marshals arguments.  Build the library in-tree first:
``python -m paper_1705_08019_amd.build``.
"""
from ._lib import FitError, lib  # noqa: F401
from .grid import FitGrid  # noqa: F401
from .adjoint import ProbeProblem, probe_energy  # noqa: F401
from .batch import FitBatch  # noqa: F401

__all__ = ["FitGrid", "FitBatch", "FitError", "lib", "ProbeProblem", "probe_energy"]
