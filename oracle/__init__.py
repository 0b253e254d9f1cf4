"""FP64 CPU oracle for the Randomized K-FAC K-factor pipeline.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The GPU
product path (``paper_2206_15397_amd``) never imports it and shares no code with it.

The oracle is written from the paper (Puiu, "Randomized K-FACs: Speeding up K-FAC with
Randomized Numerical Linear Algebra", arXiv 2206.15397):

* the exponential-average K-factor update (Algorithm 1, forward and backward EA lines;
  matrix form of Section 3),
* the Gaussian test matrix, range finder with power iterations, SREVD (Algorithm 3) and
  RSVD (Algorithm 2, using the V factor as Section 2.2.2 recommends),
* the damped low-rank inverse application (Section 4.1, the identity for
  (U D U^T + lambda I)^{-1} V, used by Algorithms 4 and 5),
* a cyclic Jacobi full eigendecomposition (plain C, ``jacobi.c``).

Everything is float64.  Inputs that arrive as bf16/fp32 are converted exactly.
"""
from .kfac_oracle import *  # noqa: F401,F403
