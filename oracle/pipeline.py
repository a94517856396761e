"""Block-wise 2D approximate DCT pipeline, written as plain dense integer math.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline may use this module.  It shares no code with the HIP library.

The still-image experiment of section 5.1: split the image into
non-overlapping N x N blocks A, transform each block, keep the first r
coefficients of the zig-zag scan, inverse-transform and measure PSNR.

Readings taken where the paper is silent or ambiguous:
  * 2D form.  The separable form B = T A T^T is used (b[v][u]: v is the
    vertical frequency, u the horizontal one).  Section 5.1 prints
    B = C A C^-1, which coincides with the separable form only for an
    orthogonal C; ``forward2d_paper_literal`` keeps that form for comparison.
  * Inverse.  The exact inverse A = T^-1 B T^-T is used (sections 3 and 6.1
    give it as a fast algorithm).  With U = N T^-1 (an integer matrix) the
    reconstruction is X / N^2 with X = U B U^T.  Because the diagonal scale S
    commutes with an element-wise mask, S cancels under zonal retention and
    the integer path never needs it.
  * Level shift and rounding.  8-bit input is shifted by -128 before the
    forward transform (JPEG convention).  The reconstruction is
    round(X / N^2) with the paper's round() (half away from zero, section 3),
    then +128 and clipped to [0, 255].  16-bit residual input is not shifted
    and its reconstruction saturates to int16.
  * Zig-zag.  The JPEG scan (the paper cites Wallace), generalised to N x N
    by anti-diagonals; the same rule is used for N = 16 and 32.
  * Quantisation (section 3.1 says S can be absorbed into the quantiser; the
    paper fixes no quantiser).  The orthonormal coefficient c = s_v s_u b is
    quantised with a uniform step Q, written in fixed point:
        g_vu  = Q * sqrt(d_v * d_u)          (d = diag(T T^T), float64)
        MQ_vu = round(2^24 / g_vu)            level = sign(b) * ((|b| MQ + 2^23) >> 24)
        DQ_vu = round(2 * g_vu)               b~ = level * DQ   (1 fractional bit)
    and the reconstruction is round(X / (2 N^2)) with X = U b~ U^T.  One
    fractional bit keeps every intermediate of a 32-point inverse within
    32-bit integers for steps up to 4096.
  * PSNR uses peak 255 and the whole-image MSE; +inf when SSE = 0.
"""
from __future__ import annotations

import math

import numpy as np

from .matrices import (dct2_matrix, diag_ttt, scale_vector, scaled_inverse, transform_matrix,
                       zigzag, near_orthogonal)
from .metrics import coding_gain_2d, variance_from_sums

QUANT_SHIFT = 24          # fixed-point bits of the forward quantiser multiplier
QUANT_FRAC = 1            # fractional bits carried by the dequantised coefficient


def round_half_away_div(p: np.ndarray, q: int) -> np.ndarray:
    """round(p / q) for integer p and positive integer q, with the paper's
    round() (half away from zero), in exact integer arithmetic.
    Section 3: the paper's round()."""
    p = np.asarray(p, dtype=np.int64)
    mag = (2 * np.abs(p) + q) // (2 * q)
    return np.where(p < 0, -mag, mag)


def round_half_away_float(x: np.ndarray) -> np.ndarray:
    """The paper's round(x) = sign(x) floor(|x| + 1/2) on float64 values.  Section 3."""
    x = np.asarray(x, dtype=np.float64)
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def to_tiles(img: np.ndarray, n: int) -> np.ndarray:
    """(H, W) -> (H/N, W/N, N, N); tile (by, bx) covers rows by*N.., cols bx*N..
    Section 5.1: the non-overlapping N x N blocks."""
    h, w = img.shape
    if h % n or w % n:
        raise ValueError(f"image {h}x{w} is not a multiple of N={n}")
    return img.reshape(h // n, n, w // n, n).transpose(0, 2, 1, 3)


def from_tiles(t: np.ndarray) -> np.ndarray:
    """Section 5.1: blocks back to the image."""
    th, tw, n, _ = t.shape
    return t.transpose(0, 2, 1, 3).reshape(th * n, tw * n)


def level_shift(img: np.ndarray) -> np.ndarray:
    """uint8 pixels -> pixel - 128 (int64); int16 residuals unchanged.
    Section 5.1 (JPEG-like compression; the JPEG level shift)."""
    if img.dtype == np.uint8:
        return img.astype(np.int64) - 128
    if img.dtype == np.int16:
        return img.astype(np.int64)
    raise TypeError(f"unsupported pixel type {img.dtype}")


def forward2d(img: np.ndarray, kind: int, n: int) -> np.ndarray:
    """b = T A T^T for every tile; returns int64 (H/N, W/N, N, N).
    Section 5.1: the 2D transform of each block."""
    t = transform_matrix(kind, n)
    a = to_tiles(level_shift(img), n)
    return t @ a @ t.T


def forward2d_paper_literal(img: np.ndarray, kind: int, n: int) -> np.ndarray:
    """B = C A C^-1 with C = S' T (section 5.1 as printed), float64."""
    c = near_orthogonal(kind, n)
    a = to_tiles(level_shift(img), n).astype(np.float64)
    return c @ a @ np.linalg.inv(c)


def zigzag_mask(n: int, r: int) -> np.ndarray:
    """Boolean (N, N) mask of the first r zig-zag positions.  Section 5.1: zonal retention."""
    if not 0 <= r <= n * n:
        raise ValueError("r out of range")
    m = np.zeros((n, n), dtype=bool)
    for v, u in zigzag(n)[:r]:
        m[v, u] = True
    return m


def zigzag_gather(b: np.ndarray, r: int) -> np.ndarray:
    """First r coefficients of each tile in zig-zag order: (..., r).
    Section 5.1: zonal retention."""
    n = b.shape[-1]
    zz = zigzag(n)[:r]
    vs = np.array([v for v, _ in zz], dtype=np.int64)
    us = np.array([u for _, u in zz], dtype=np.int64)
    return b[..., vs, us]


def zigzag_scatter(kept: np.ndarray, n: int) -> np.ndarray:
    """Inverse of ``zigzag_gather``: zero-filled (..., N, N) tiles.
    Section 5.1: zonal retention."""
    r = kept.shape[-1]
    out = np.zeros(kept.shape[:-1] + (n, n), dtype=kept.dtype)
    for i, (v, u) in enumerate(zigzag(n)[:r]):
        out[..., v, u] = kept[..., i]
    return out


def retain(b: np.ndarray, r: int) -> np.ndarray:
    """Zonal retention: zero every coefficient outside the first r zig-zag
    positions (section 5.1)."""
    n = b.shape[-1]
    return np.where(zigzag_mask(n, r), b, 0)


def scaled_coefficients(b: np.ndarray, kind: int, n: int) -> np.ndarray:
    """c_vu = s_v s_u b_vu: coefficients of the near-orthogonal C = S' T, float64.
    Section 3.1: the orthogonalising scale."""
    s = scale_vector(kind, n)
    return np.outer(s, s) * b.astype(np.float64)


def quant_tables(kind: int, n: int, qstep: int):
    """(MQ, DQ) int64 (N, N) tables of the fixed-point quantiser."""
    d = diag_ttt(kind, n).astype(np.float64)
    g = qstep * np.sqrt(np.outer(d, d))
    mq = round_half_away_float(float(1 << QUANT_SHIFT) / g).astype(np.int64)
    dq = round_half_away_float(float(1 << QUANT_FRAC) * g).astype(np.int64)
    return mq, dq


def quantise(b: np.ndarray, mq: np.ndarray) -> np.ndarray:
    """level = sign(b) * floor(|b| MQ / 2^24 + 1/2)  (int64).
    Section 3.1 lets S be absorbed in a quantiser; this one is the project's own (parity
    unpinned against the paper)."""
    b = np.asarray(b, dtype=np.int64)
    mag = (np.abs(b) * mq + (1 << (QUANT_SHIFT - 1))) >> QUANT_SHIFT
    return np.where(b < 0, -mag, mag)


def dequantise(level: np.ndarray, dq: np.ndarray) -> np.ndarray:
    """The inverse step of ``quantise`` (section 3.1; parity unpinned against the paper)."""
    return np.asarray(level, dtype=np.int64) * dq


def inverse2d(b: np.ndarray, kind: int, n: int, out_dtype, frac_bits: int = 0) -> np.ndarray:
    """Reconstruct an image from (H/N, W/N, N, N) integer coefficients.

    X = U b U^T with U = N T^-1, y = round(X / (2^frac_bits N^2)); 8-bit output
    adds 128 and clips to [0, 255], 16-bit output saturates.
    Section 5.1 with the exact inverse of sections 3 and 6.1.
    """
    u = scaled_inverse(kind, n)
    x = u @ np.asarray(b, dtype=np.int64) @ u.T
    y = from_tiles(round_half_away_div(x, (1 << frac_bits) * n * n))
    if np.dtype(out_dtype) == np.uint8:
        return np.clip(y + 128, 0, 255).astype(np.uint8)
    if np.dtype(out_dtype) == np.int16:
        return np.clip(y, -32768, 32767).astype(np.int16)
    raise TypeError(f"unsupported output type {out_dtype}")


def sse(a: np.ndarray, b: np.ndarray) -> int:
    """Section 5.1: the squared error behind the PSNR."""
    d = a.astype(np.int64) - b.astype(np.int64)
    return int(np.sum(d * d))


def psnr(sse_value: int, num_pixels: int, peak: float = 255.0) -> float:
    """PSNR = 10 log10(peak^2 / MSE) in float64; +inf when SSE = 0.
    Section 5.1: quality measured by PSNR."""
    if sse_value == 0:
        return math.inf
    mse = sse_value / float(num_pixels)
    return 10.0 * math.log10(peak * peak / mse)


def compress(img: np.ndarray, kind: int, n: int, r: int, qstep: int = 0) -> dict:
    """The whole pipeline of one image.

    qstep = 0: zonal retention of the first r zig-zag coefficients.
    qstep > 0: the first r zig-zag coefficients are quantised with step qstep
    (r = N^2 quantises every coefficient).

    Returns a dict with
      ``kept``   int64 (H/N, W/N, r): retained coefficients (or levels) in zig-zag order
      ``scaled`` float64 (H/N, W/N, r): s_v s_u b_vu of the retained positions
      ``recon``  reconstruction, same dtype and shape as ``img``
      ``sse``    exact sum of squared reconstruction errors
      ``psnr``   float64
    Section 5.1: the JPEG-like experiment for one image.
    """
    b = forward2d(img, kind, n)
    scaled = zigzag_gather(scaled_coefficients(b, kind, n), r)
    if qstep == 0:
        kept = zigzag_gather(b, r)
        recon = inverse2d(zigzag_scatter(kept, n), kind, n, img.dtype)
    else:
        mq, dq = quant_tables(kind, n, qstep)
        levels = retain(quantise(b, mq), r)
        kept = zigzag_gather(levels, r)
        recon = inverse2d(dequantise(levels, dq), kind, n, img.dtype, QUANT_FRAC)
    e = sse(img, recon)
    return dict(kept=kept, scaled=scaled, recon=recon, sse=e,
                psnr=psnr(e, img.size))


def coefficient_moments(img: np.ndarray, kind: int, n: int) -> dict:
    """Per-image sums behind the empirical coding gain: over the tiles of
    ``img``, the sum and the sum of squares of every integer coefficient
    b[v][u] of B = T A T^T (``s1``, ``s2``: Python-int (N, N) object arrays),
    and over the pixels a of A (level-shifted for 8-bit input) their sum and
    sum of squares (``a1``, ``a2``); ``tiles`` and ``pixels`` count them.
    Sections 4.1 and 5.1."""
    b = forward2d(img, kind, n).reshape(-1, n, n)
    a = level_shift(img)
    s1 = np.empty((n, n), dtype=object)
    s2 = np.empty((n, n), dtype=object)
    for v in range(n):
        for u in range(n):
            col = b[:, v, u].astype(object)
            s1[v, u] = int(sum(col))
            s2[v, u] = int(sum(x * x for x in col))
    av = a.reshape(-1).astype(object)
    return dict(tiles=b.shape[0], s1=s1, s2=s2, pixels=a.size, a1=int(sum(av)),
                a2=int(sum(x * x for x in av)))


def coefficient_variances(mom: dict, kind: int, n: int):
    """(var_c, var_x): the variance over the tiles of every scaled coefficient
    c_vu = s_v s_u b_vu, and the variance of the pixels, from the sums of
    ``coefficient_moments``.  Section 3.1 (the scale) and section 4.1."""
    s = scale_vector(kind, n)
    var_b = np.array([[variance_from_sums(mom["tiles"], mom["s1"][v, u], mom["s2"][v, u])
                       for u in range(n)] for v in range(n)])
    var_x = variance_from_sums(mom["pixels"], mom["a1"], mom["a2"])
    return np.outer(s * s, s * s) * var_b, var_x


def empirical_coding_gain(img: np.ndarray, kind: int, n: int, basis: str = "cols") -> float:
    """2D unified coding gain (dB) of C = S' T measured on one image: the
    coefficient and pixel variances over its tiles in place of the AR(1)
    model's.  Section 4.1, extended to the separable 2D transform of
    section 5.1."""
    var_c, var_x = coefficient_variances(coefficient_moments(img, kind, n), kind, n)
    return coding_gain_2d(near_orthogonal(kind, n), var_c, var_x, basis)


# ----------------------------------------------- the exact DCT (section 5.1)
def compress_dct(img: np.ndarray, r: int) -> dict:
    """The still-image experiment with the exact 8-point DCT-II, the reference
    transform of section 5 (float64): c = C A C^T with the orthonormal C8,
    the first r zig-zag coefficients kept, A~ = C^T c C, then round, +128
    and clip (or saturate for int16).  ``scaled`` holds the kept orthonormal
    coefficients in zig-zag order; ``margin`` is each pixel's distance from
    the nearest rounding tie (A~ + 1/2 at an integer), which says where a
    reconstruction in lower precision may round the other way."""
    n = 8
    c8 = dct2_matrix(n)
    a = to_tiles(level_shift(img), n).astype(np.float64)
    coef = c8 @ a @ c8.T
    scaled = zigzag_gather(coef, r)
    masked = np.where(zigzag_mask(n, r), coef, 0.0)
    x = from_tiles(c8.T @ masked @ c8)
    y = round_half_away_float(x)
    frac = np.abs(x) - np.floor(np.abs(x))
    margin = np.abs(frac - 0.5)
    if img.dtype == np.uint8:
        recon = np.clip(y + 128, 0, 255).astype(np.uint8)
    else:
        recon = np.clip(y, -32768, 32767).astype(np.int16)
    e = sse(img, recon)
    return dict(scaled=scaled, recon=recon, sse=e, psnr=psnr(e, img.size), margin=margin)
