"""CPU oracle for the randomized row-leverage-score (rSLS) estimator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the tests, the smoke check in
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use
it.  It shares no code with the HIP library and imports nothing from it.

Everything here is plain, slow and written to be checked by eye against the
paper (Sobczyk & Gallopoulos, "Estimating leverage scores via rank revealing
methods and randomization"):

* ``conventions`` -- the random objects the paper leaves unspecified (hash
  family of the CountSketch, the sign polynomial, the Gaussian generator),
  each written from its published definition.
* ``leverage`` -- exact leverage scores (plain definitions, Section 1) and
  the estimator LS-HRN-approx (Algorithm 10 = Algorithm 4 + Algorithm 8),
  step by step in FP64.
* ``gradient`` -- the reference gradient of w^T theta~ at a fixed sketch.
"""

from . import conventions, leverage  # noqa: F401
