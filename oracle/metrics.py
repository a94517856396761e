"""Assessment measures of sections 3.1 and 4, in float64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline may use this module.  It shares no code with the HIP library.

  * deviation from diagonality delta(M) (section 3.1);
  * total error energy eps = pi ||C - C^||_F^2 (section 4.1, Table 1);
  * unified coding gain C_g and the KLT coding gain under the AR(1) model
    R_x[m][n] = rho^|m-n| (section 4.1);
  * additive complexity of a chain of sparse factors (section 4.2, Tables 2
    and 4).

Reading: section 4.1 defines g_k as the k-th row of C^-1.  The textbook
unified coding gain uses the synthesis basis, i.e. the columns of C^-1.  Both
agree for orthogonal C.  ``coding_gain(..., basis="rows")`` follows the
paper literally and ``basis="cols"`` gives the textbook form; the values for
the proposed non-orthogonal transforms are parity unpinned (the figure that
could separate the two readings is missing from the paper).
"""
from __future__ import annotations

import math

import numpy as np


def deviation_from_diagonality(m: np.ndarray) -> float:
    """Section 3.1: the deviation from diagonality."""
    m = np.asarray(m, dtype=np.float64)
    return 1.0 - float(np.sum(np.diag(m) ** 2)) / float(np.sum(m * m))


def total_error_energy(c_exact: np.ndarray, c_approx: np.ndarray) -> float:
    """Section 4.1: the total error energy (Table 1)."""
    d = np.asarray(c_exact, np.float64) - np.asarray(c_approx, np.float64)
    return math.pi * float(np.sum(d * d))


def ar1_covariance(n: int, rho: float) -> np.ndarray:
    """Section 4.1: the first-order Markov model."""
    idx = np.arange(n)
    return rho ** np.abs(idx[:, None] - idx[None, :]).astype(np.float64)


def coding_gain(c: np.ndarray, rho: float, basis: str = "rows") -> float:
    """C_g = 10 log10 prod_k (A_k B_k)^(-1/N) in dB.

    A_k = su[(h_k^T h_k) o R_x] with h_k the k-th row of C; B_k = ||g_k||^2
    with g_k the k-th row (basis="rows") or column (basis="cols") of C^-1.
    Section 4.1: the coding gain.
    """
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    r = ar1_covariance(n, rho)
    cinv = np.linalg.inv(c)
    g = cinv if basis == "rows" else cinv.T
    total = 0.0
    for k in range(n):
        h = c[k]
        a_k = float(np.sum(np.outer(h, h) * r))
        b_k = float(np.dot(g[k], g[k]))
        total += math.log10(a_k * b_k)
    return -10.0 * total / n


def klt_coding_gain(n: int, rho: float) -> float:
    """Coding gain of the KLT: the eigenvalues of R_x are its subband variances.  Section 4.1."""
    lam = np.linalg.eigvalsh(ar1_covariance(n, rho))
    return -10.0 * float(np.mean(np.log10(lam)))


def additions_of_factor(m: np.ndarray) -> int:
    """Additions needed to apply a sparse factor whose non-zero entries are
    +-1 or powers of two: each output row with k non-zeros costs k - 1 additions
    (sign changes and power-of-two scalings are free).
    Section 4.2: addition counts (Tables 2 and 4)."""
    m = np.asarray(m)
    return int(sum(max(int(np.count_nonzero(row)) - 1, 0) for row in m))


def additions_of_chain(factors) -> int:
    """Section 4.2: addition counts (Tables 2 and 4)."""
    return sum(additions_of_factor(f) for f in factors)
