"""Oracle for the exact multivariate polynomial determinant (test infrastructure only).

This package is a plain, slow, CPU-only restatement of what the GPU path computes, written
from the paper (Wei & Chen, "Optimized Multivariate Polynomial Determinant on GPU",
arXiv 2010.12117) and from the textbook definitions it relies on. Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it; the product path
never does.

Modules
-------
poly      dense multivariate polynomials over Z as exponent-tuple dicts, the input
          encoding of the paper's Section 2 (FFT paragraph, the worked example
          F = 1 + 2x + 3xy + 4x^2 + 5y^2), exact multivariate division.
det       the determinant by definition (Leibniz permutation expansion), fraction-free
          Bareiss elimination over Z[x1..xk] ("oracle A"), Gaussian elimination over Q
          with fractions, and pointwise integer Bareiss with exact interpolation on the
          integer grid ("oracle B").
plan      the plan quantities of Section 2: per-variable degree bound of the determinant,
          power-of-two grid (the example (15,7,9) -> (16,8,16)), the coefficient bound and
          the number of primes, NTT primes of the form c*2^q+1 (equation "primes").
modular   the modular method of Algorithm 1 step by step, for small inputs: reduction,
          evaluation at roots of unity (Section 2, DFT over Z/pZ), determinant mod p,
          interpolation by the inverse transform (Section 3.3), and mixed-radix
          conversion (Section 3.4, Algorithm 4) plus plain CRT for cross-checks.
"""
