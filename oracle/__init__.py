"""CPU oracle for TT multigroup radiation transport.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and
this package never imports the GPU library.

* ``planck``: group emission coefficients by mpmath quadrature (Section 2).
* ``dense``:  dense FP64 full-grid march in plain C + OpenMP (Section 2.1).
* ``tt``:     explicit TT-sum apply (Appendix A) and Oseledets TT-SVD rounding
              (the SVD rounding method the paper cites), in numpy FP64.

Parity pins live in tests/test_oracle_*.py; every function here is pinned by
a closed form, a brute-force or library check, or a value the paper prints.
"""
from . import planck, dense, tt  # noqa: F401


def build(force: bool = False):
    """Compile the C part of the oracle (gcc + OpenMP)."""
    return dense.build(force=force)
