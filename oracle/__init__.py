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
  metrics   -- deviation from diagonality, total error energy, coding gain
               (the AR(1) closed form and the 2D form from measured
               variances), addition counts (sections 3.1, 4)

Parity status: every function is pinned by the tests under ``tests/``
against values the paper prints, closed forms or brute force, except
  * the fixed-point quantiser (the paper defines none): parity unpinned
    against the paper, pinned only against the float64 uniform quantiser it
    approximates;
  * the coding gain of the non-orthogonal transforms: the columns reading of
    g_k is pinned by the paper's description of its coding-gain figure (the
    figure itself is missing), the rows reading only by the DCT/KLT values
    the paper prints;
  * the empirical 2D coding gain: pinned against the AR(1) model's
    population moments (exactly twice the 1D gain) and, statistically, on a
    large synthetic field; the paper defines only the model's closed form;
  * the SSIM of section 5.1: pinned by closed forms (identical and constant
    images), symmetry and a brute-force window, but parity unpinned against
    the paper's own SSIM values, whose images are not available.
"""
from . import matrices, metrics, pipeline  # noqa: F401
