"""CPU oracle for randomized block-Krylov tensor-train approximation (TT-RBKI).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package.  The GPU
library never calls it, links it or reads its outputs, and the two share no
code: the only common dependency is the seeded input generator module
``synth`` (which holds none of the method's arithmetic).

Everything here is plain, slow, float64 numpy, written from arXiv:2308.01480:

* ``philox``  -- the Gaussian test matrix Omega drawn by the method, from the
  published Philox4x64-10 counter-based generator (Salmon et al., SC'11) and
  the Box-Muller transform.
* ``ttrbki``  -- TT-SVD (Algorithm 1, fixed-rank and delta-truncated) and
  TT-RBKI (Algorithm 3, in the column-space block-Krylov form with
  Rayleigh-Ritz truncation), mode by mode in the paper's order.
* ``metrics`` -- relative error and PSNR (Section 4), tail energy
  (Definition 3), reconstruction, TT inner products and principal angles.

Pins (tests/test_oracle_*.py) tie these to things other than themselves:
numpy's own Philox implementation, LAPACK SVDs of every processed unfolding,
exact low-TT-rank reconstruction, Theorem 1's bound, the tail identity of
TT-SVD, the closed-form error of an orthogonally decomposable tensor, the
Pythagorean identity behind Eq. (12), and Ky Fan / nestedness properties.
"""
from . import philox, ttrbki, metrics  # noqa: F401
