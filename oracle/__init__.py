"""FP64 CPU oracle for sparse-correlation orientation matching (ACOM).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constants) and is written from
the paper (Ophus et al., "Automated crystal orientation mapping in py4DSTEM
using sparse correlation matching", arXiv 2111.00171) as plain, slow,
obviously-correct FP64 NumPy (plus one plain-C direct sum for speed).

Modules
  crystal   reciprocal basis, reflection list, structure factors   (Methods: Structure Factor Calculations)
  zones     SLERP zone-axis grid, zone rotation matrices           (Methods: Generation of an Orientation Plan, Eq. rotation_matrices)
  plan      excitation error, orientation plan P0, normalisation   (Methods: Kinematical Diffraction; Orientation Plan)
  image     sparse polar image X                                   (Methods: Correlation Pattern Matching, Eq. image_polar)
  correlate direct-sum correlogram, FFT route, decisions           (Methods: Correlation Pattern Matching)
  kinematics forward kinematical pattern (for pins)                (Methods: Calculation of Kinematical Diffraction Patterns)
  score     continuous Gaussian score, gradient, refinement        (extension; see module docstring)
  metrics   misorientation / zone-axis error                       (Results: kinematical and dynamical tests)
  directsum plain-C FP64 direct sum over many patterns (ctypes)

Every function names the passage of the paper it follows.  Where the paper is
silent or ambiguous the reading taken is stated in the docstring; functions
without an independent pin say "parity unpinned".
"""
from . import crystal, zones, plan, image, correlate, kinematics, score, metrics  # noqa: F401
