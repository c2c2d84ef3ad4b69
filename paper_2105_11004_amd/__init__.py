"""MI355X-native randomized row-leverage-score (rSLS) estimator.

The compute path lives in the HIP library ``liblev.so`` (sources under
``csrc/``, C interface in ``include/lev.h``).  This package is a thin
ctypes binding over it (``api``, which also holds ``LevEstimate``, the
``torch.autograd.Function`` over the hand-written adjoint), the build step
(``build``) and the seeded synthetic workloads used by the tests and the
benchmark (``workloads``).  Importing the package does
not load the library; the first call into ``api`` does, and raises if the
library is missing -- there is no CPU fallback.
"""

__all__ = ["api", "workloads"]
