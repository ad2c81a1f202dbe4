"""FP64 CPU oracle for the sketch-and-solve null-space method (Algorithm 1 of Park & Nakatsukasa).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.  The
library under ``paper_2206_00975_amd`` never imports it, and this package imports nothing
from the library: the two share no code, tables or constants.

What the oracle computes, plainly and slowly, with every floating-point step in FP64:

* ``philox``    -- the Philox4x32-10 counter-based generator (Salmon et al., SC'11), written
                   from its published definition.
* ``draws``     -- the random objects the sketches are built from: sign diagonal ``D``,
                   sampled rows ``R`` (Floyd sampling without replacement), sparse-sign
                   column supports and signs, Gaussian entries (Box-Muller).
* ``operators`` -- the explicit sketch matrix ``S`` (s x m), built in column blocks, and
                   ``SA = S A`` by plain matrix products (Section 2: Gaussian ``G/sqrt(s)``,
                   subsampled randomized trigonometric transform, sparse sign).
* ``svd``       -- plain one-sided (Hestenes) Jacobi SVD of ``SA`` itself, no QR.
* ``updates``   -- row updates and downdates of a sketch (Section 5, Algorithms 2 and 3).
* ``aaa``       -- AAA rational approximation with a reused, updated sketch (Section 6).
* ``method``    -- Algorithm 1 (trailing right singular vectors), total least squares
                   (Section 4) and the gradient of a TLS loss through the sketch.
* ``metrics``   -- canonical-angle sines (Definition 3.1), residual ratios (Table 1),
                   the relative gap chi and the bounds of Theorems 2.3 and 3.2.

Parity status (which functions have an external pin) is listed in each module header.
"""
