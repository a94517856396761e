"""Assessment measures of sections 3.1 and 4, in float64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline may use this module.  It shares no code with the HIP library.

  * deviation from diagonality delta(M) (section 3.1);
  * total error energy eps = pi ||C - C^||_F^2 (section 4.1, Table 1);
  * unified coding gain C_g and the KLT coding gain under the AR(1) model
    R_x[m][n] = rho^|m-n| (section 4.1);
  * additive complexity of a chain of sparse factors (section 4.2, Tables 2
    and 4);
  * the structural similarity index SSIM (Gaussian 11 x 11 window, sigma 1.5,
    K1 = 0.01, K2 = 0.03, mean over every full window) and the absolute
    percentage error relative to the exact DCT, the image-quality measures of
    section 5.1.  The paper cites the SSIM without restating it; the index
    is taken as its authors define it, without any downsampling.  Pinned by
    closed forms (identical images, constant images), symmetry and a
    brute-force window; parity unpinned against the paper's own SSIM values,
    whose images are not available.

Reading: section 4.1 defines g_k as the k-th row of C^-1.  The textbook
unified coding gain uses the synthesis basis, i.e. the columns of C^-1.  Both
agree for orthogonal C.  ``coding_gain(..., basis="rows")`` follows the
paper literally and ``basis="cols"`` gives the textbook form.  The figure of
section 4.1 is missing, but the text describes it: the DCT is closest to the
KLT, followed by HT and WHT (equal), the proposed transforms beat SDCT, and as
rho -> 1 the round-based C^8 performs as well as HT and WHT.  Only the
columns reading satisfies that description: with rows, C^8 overtakes WHT
from rho ~ 0.95 on and ends 0.06 dB above it, while with columns it stays
below WHT and meets it within 0.002 dB as rho -> 1.  The tests pin the
columns reading to those statements; the rows reading is kept for
comparison.

Empirical 2D coding gain (an addition for measured images; the paper gives
only the AR(1) closed form): for a separable 2D transform the synthesis
basis image of coefficient (v, u) is g_v g_u^T, with squared norm
B_v B_u, and A_vu is the variance of the scaled coefficient c_vu relative
to the pixel variance.  Under the separable AR(1) model the coefficient
variances are (C R C^T)_vv (C R C^T)_uu, so the 2D gain is exactly twice
the 1D gain; the tests pin ``coding_gain_2d`` to that.
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


def synthesis_norms(c: np.ndarray, basis: str = "rows") -> np.ndarray:
    """B_k = ||g_k||^2 for every k, g_k the k-th row (basis="rows") or column
    (basis="cols") of C^-1.  Section 4.1: the coding gain's B_k."""
    cinv = np.linalg.inv(np.asarray(c, dtype=np.float64))
    g = cinv if basis == "rows" else cinv.T
    return np.einsum("kj,kj->k", g, g)


def coding_gain_2d(c: np.ndarray, var_c: np.ndarray, var_x: float, basis: str = "rows") -> float:
    """2D unified coding gain of the separable transform c (x) c, in dB:
    -10/N^2 sum_{v,u} log10(A_vu B_v B_u) with A_vu = var_c[v][u] / var_x, the
    variance of coefficient (v, u) of C A C^T relative to the pixel variance.
    +inf if some coefficient has zero variance and the pixels do not; NaN if
    the pixel variance is zero.  Section 4.1 (the unified coding gain), extended
    to the separable 2D transform."""
    var_c = np.asarray(var_c, dtype=np.float64)
    n = var_c.shape[0]
    if var_x == 0:
        return math.nan
    if np.any(var_c == 0):
        return math.inf
    b = synthesis_norms(c, basis)
    total = 0.0
    for v in range(n):
        for u in range(n):
            total += math.log10(var_c[v, u] / var_x * b[v] * b[u])
    return -10.0 * total / (n * n)


def variance_from_sums(count: int, s1: int, s2: int) -> float:
    """Population variance (s2 - s1^2 / count) / count of ``count`` integers
    with sum s1 and sum of squares s2, evaluated exactly and rounded once."""
    from fractions import Fraction
    return float(Fraction(int(count) * int(s2) - int(s1) * int(s1), int(count) * int(count)))


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


# ------------------------------------------------ structural similarity (SSIM)
SSIM_WINDOW = 11          # Gaussian window of the SSIM index, 11 x 11
SSIM_SIGMA = 1.5          # its standard deviation
SSIM_K1, SSIM_K2 = 0.01, 0.03


def ssim_window() -> np.ndarray:
    """The normalised 11 x 11 Gaussian weighting window (sigma 1.5) of the
    SSIM index that section 5.1 cites (Wang et al. 2004)."""
    r = SSIM_WINDOW // 2
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(t[:, None] ** 2 + t[None, :] ** 2) / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def ssim_map(x: np.ndarray, y: np.ndarray, peak: float = 255.0) -> np.ndarray:
    """SSIM of every full 11 x 11 window of two images (the 'valid' windows,
    (H - 10) x (W - 10) of them), in float64:
      SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))
    with Gaussian-weighted means, variances and covariance and
    C1 = (K1 L)^2, C2 = (K2 L)^2.  Section 5.1's quality measure (Wang et
    al. 2004), evaluated window by window as a weighted sum."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = ssim_window()
    k = SSIM_WINDOW
    h, wd = x.shape
    if h < k or wd < k:
        raise ValueError("images smaller than the SSIM window")
    c1 = (SSIM_K1 * peak) ** 2
    c2 = (SSIM_K2 * peak) ** 2
    from numpy.lib.stride_tricks import sliding_window_view
    xw = sliding_window_view(x, (k, k))
    yw = sliding_window_view(y, (k, k))
    mx = np.einsum("ijab,ab->ij", xw, w)
    my = np.einsum("ijab,ab->ij", yw, w)
    sxx = np.einsum("ijab,ab->ij", (xw - mx[..., None, None]) ** 2, w)
    syy = np.einsum("ijab,ab->ij", (yw - my[..., None, None]) ** 2, w)
    sxy = np.einsum("ijab,ab->ij", (xw - mx[..., None, None]) * (yw - my[..., None, None]), w)
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx ** 2 + my ** 2 + c1) * (sxx + syy + c2))


def mean_ssim(x: np.ndarray, y: np.ndarray, peak: float = 255.0) -> float:
    """Mean SSIM over all full windows (section 5.1's SSIM of an image pair)."""
    return float(np.mean(ssim_map(x, y, peak)))


def absolute_percentage_error(value: float, reference: float) -> float:
    """APE of a measure relative to the exact DCT's (section 5.1), in percent."""
    return 100.0 * abs(value - reference) / abs(reference)
