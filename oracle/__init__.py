"""CPU oracle for the block-wise Chen-based approximate DCT.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, dense reference
implementation that the HIP library is checked against.  Only the tests, the
``smoke()`` check and the benchmark's ``cpu_baseline`` leg may import it; the
library never does, and the two share no code (the synthetic input generators
live in the separate ``synth`` module, which holds no transform arithmetic).

Modules:
  matrices  -- transform matrices from the paper's factorizations (sections 2,
               3, 3.1, 6.1), exact inverses, scale factors, zig-zag order
  pipeline  -- tile transform, retention, quantisation, inverse, PSNR
               (sections 3.1, 5.1)
  metrics   -- deviation from diagonality, total error energy, coding gain,
               addition counts (sections 3.1, 4)

Parity status: every function is pinned by the tests under ``tests/``
against values the paper prints, closed forms or brute force, except
  * the fixed-point quantiser (the paper defines none): parity unpinned
    against the paper, pinned only against the float64 uniform quantiser it
    approximates;
  * the coding gain of the non-orthogonal transforms under the two readings
    of g_k: parity unpinned beyond the DCT/KLT values the paper prints.
"""
from . import matrices, metrics, pipeline  # noqa: F401
