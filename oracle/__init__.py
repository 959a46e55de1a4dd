"""CPU FP64 oracle for FEF pair energies and the effective-field SCF.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package.  It shares no code
with the HIP library or its Python binding, and imports neither.

Every function states the plain definition it writes out and the passage of
the paper it follows (arXiv:1708.03377, "Computing solvated excited states
using fragment-effective-field coupled-cluster perturbation theory").
"""
from . import fef, mlp  # noqa: F401
