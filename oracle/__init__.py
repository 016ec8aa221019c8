"""Reference (oracle) implementation of the adaptive product-convolution
approximation of Alger, Rao, Myers, Bui-Thanh and Ghattas (arXiv 1805.06018).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation written from the paper's definitions.  It exists to check the
HIP library; it is never used by the library itself.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the HIP path: no kernels, headers, tables or helpers.

Modules
  grid       sample points, cells(p), blocky neighbourhoods U_k, nbrs(k)  (Sec. 2.2)
  weights    harmonic partition-of-unity weights w_k                     (Sec. 2.4)
  extension  extended impulse responses phi_k^E                          (Sec. 2.5)
  apply      A~ f = sum_k phi_k^E * (w_k . f), its adjoint, matrix entries (eq. (2.5)/(1.6), Sec. 3)
  estimator  randomized a-posteriori estimator eta_C                     (Sec. 2.6)
  direct     ctypes wrapper of a plain C direct-summation core (same sums,
             used where NumPy loops are too slow)

Every part is pinned by the tests against worked values, closed forms and
brute force; the extension with neighbours supplied on boxes of unequal radii
by hand-derived values (tests/golden/extension_unequal_radii.txt).
"""
from .grid import Grid, TilingError
from .weights import harmonic_weights, leaf_weights
from .extension import extended_kernels
from .apply import OracleOperator
from .estimator import estimate

__all__ = ["Grid", "TilingError", "harmonic_weights", "leaf_weights",
           "extended_kernels", "OracleOperator", "estimate"]
