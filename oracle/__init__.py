"""CPU oracle for the full-rank-Cholesky Moore-Penrose inverse.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or
executes this package; only the tests, the package smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU path.

* ``geninv_ref`` -- float64 NumPy implementation of the paper's algorithm,
  step by step (Gram, tolerance, full-rank Cholesky, (L'L)^-1, product chain)
  plus least squares, the Penrose error measures, the rounding-sensitivity
  and decision-band checkers, and the Newton-Schulz refinement step.
* ``exact``      -- exact rational pseudoinverse of tiny integer matrices by
  an independent formula, used to pin ``geninv_ref``.
* ``ozaki_ref``  -- float64/integer reference of the fixed-point column
  slicing and sliced products used by the mixed-precision form.
* ``crt_ref``    -- reference of the int8 engine's products: the exact
  product of fixed-point integer representations, rounded once.
"""
from . import geninv_ref, exact  # noqa: F401
