"""FP64 CPU oracle for the SARABANDE 3/4PCF hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the entry module
and the CPU-baseline leg of the bench may import this package.  The product
library never does, and this package imports nothing from it.

The oracle is the plain definition of what the method computes (Sec. 2 of
Sunseri et al. 2022, arXiv 2210.10206), evaluated by direct real-space
correlation in float64 instead of by FFTs:

* the binned coefficients a^b_lm(x) of eq. (almconv) and c^b_m(x) of
  eqs. (discretize_cmb) and (c_m def) as explicit sums over the grid offsets of
  each radial bin;
* the grid sums of Alg. 5 (full 3PCF), Alg. 6 (full 4PCF), Alg. 7 (projected
  3PCF) and Alg. 8 (projected 4PCF), written as the full sums over m (and M)
  that those listings halve with symmetry tricks;
* the gradient of a linear functional of the full 3PCF with respect to the
  density (no counterpart in the paper; it is the derivative of the same sums).

Prefactors ((-1)^l / sqrt(2l+1), 1/(2 pi)^2, 1/V, 1/V_b) are not applied: the
returned values are the raw sums of the appendix listings.  Where the paper is
ambiguous, the reading taken is stated in the docstring of the function concerned.

Parity pins (all in ``tests/``): brute-force triplet / quadruplet counting on
tiny grids, 3j closed forms and orthogonality, rotation / reflection
invariance, the constant-field closed form, homogeneity, and finite
differences of the gradient.  Functions without an independent pin say so in
their docstring ("parity unpinned").
"""
from .api import (  # noqa: F401
    support, bin_counts, basis_full, basis_proj, lambdas, mpairs, threej,
    coeffs_full, coeffs_proj, zeta3_full, zeta4_full, zeta3_proj, zeta4_proj,
    grad3_full, normalization, max_threads,
)
