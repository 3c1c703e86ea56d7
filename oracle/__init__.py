"""Plain FP64 CPU oracle of the DQMC sweep (test infrastructure only).

This package is the correctness reference for the HIP library.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path never does.  It shares no code with the HIP path: the
only common dependency is the `inputs` package (hopping matrices and workload
parameters, no arithmetic of the method).

Everything here is deliberately plain: NumPy/SciPy FP64, one operation per
line of the paper's formulas, no blocking or fusion.  Each function cites the
section or equation of the ALF 1.0 documentation (arXiv:1704.00131) that it
follows; where the paper is silent the reading taken is stated in the
docstring.
"""
from . import philox, hubbard, stable, sweep, measure, exact_small, gradient, timedisplaced  # noqa: F401
from . import complex_field, mz_flavours, vertices  # noqa: F401
