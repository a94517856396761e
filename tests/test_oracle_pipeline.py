"""Pins of the oracle's block pipeline (section 5.1, quantiser reading of
section 3.1) against special cases with closed forms, brute force on tiny
inputs and the paper's qualitative ordering."""
from fractions import Fraction
import math

import numpy as np
import pytest

from conftest import load_matrix
from oracle import matrices as M
from oracle import pipeline as P
import synth


def rng(seed):
    return np.random.default_rng(seed)


def random_u8(h, w, seed):
    return rng(seed).integers(0, 256, size=(h, w), dtype=np.int64).astype(np.uint8)


def random_i16(h, w, seed, amp=255):
    return rng(seed).integers(-amp, amp + 1, size=(h, w)).astype(np.int16)


def printed_t8(kind):
    return load_matrix("t8_sign.txt" if kind == M.SIGN else "t8_round.txt")


# -------------------------------------------------------------- forward
@pytest.mark.parametrize("kind", M.KINDS)
def test_vertically_constant_block_gives_one_row(kind):
    # A = 1 x^T (every row equal): B = (T 1)(T x)^T = N e0 (T x)^T, with T the
    # printed matrix; a transposed operand would put the energy in column 0
    x = np.array([3, 250, 17, 128, 0, 255, 64, 90], dtype=np.uint8)
    img = np.tile(x, (8, 1))
    b = P.forward2d(img, kind, 8)[0, 0]
    t = printed_t8(kind)
    a = x.astype(np.int64) - 128
    assert np.array_equal(b[0], 8 * (t @ a))
    assert np.all(b[1:] == 0)


@pytest.mark.parametrize("kind", M.KINDS)
def test_horizontally_constant_block_gives_one_column(kind):
    x = np.array([3, 250, 17, 128, 0, 255, 64, 90], dtype=np.uint8)
    img = np.tile(x[:, None], (1, 8))
    b = P.forward2d(img, kind, 8)[0, 0]
    a = x.astype(np.int64) - 128
    assert np.array_equal(b[:, 0], 8 * (printed_t8(kind) @ a))
    assert np.all(b[:, 1:] == 0)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_constant_block_has_only_dc(kind, n):
    for c in (0, 128, 255):
        img = np.full((n, 2 * n), c, dtype=np.uint8)
        b = P.forward2d(img, kind, n)
        assert np.all(b[..., 0, 0] == n * n * (c - 128))
        b[..., 0, 0] = 0
        assert np.all(b == 0)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_level_shift_touches_dc_only(kind, n):
    img = random_u8(n, n, 1) // 2
    b0 = P.forward2d(img, kind, n)
    b1 = P.forward2d(img + 1, kind, n)
    d = b1 - b0
    assert d[0, 0, 0, 0] == n * n
    d[0, 0, 0, 0] = 0
    assert np.all(d == 0)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_transpose_equivariance(kind, n):
    img = random_u8(2 * n, 3 * n, 2)
    b = P.forward2d(img, kind, n)
    bt = P.forward2d(np.ascontiguousarray(img.T), kind, n)
    assert np.array_equal(bt, b.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("kind", M.KINDS)
def test_forward_brute_force_kronecker(kind):
    # vec(B) = (T kron T) vec(A), evaluated with Python integers
    t = printed_t8(kind).tolist()
    img = random_u8(8, 16, 3)
    b = P.forward2d(img, kind, 8)
    for bx in range(2):
        a = [[int(img[i, bx * 8 + j]) - 128 for j in range(8)] for i in range(8)]
        for v in range(8):
            for u in range(8):
                s = sum(t[v][i] * t[u][j] * a[i][j] for i in range(8) for j in range(8))
                assert b[0, bx, v, u] == s


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_scaled_coefficients_are_those_of_C_A_Ct(kind, n):
    img = random_u8(n, n, 4)
    c = M.near_orthogonal(kind, n)
    a = P.level_shift(img).astype(np.float64)
    want = c @ a @ c.T
    got = P.scaled_coefficients(P.forward2d(img, kind, n), kind, n)[0, 0]
    assert np.allclose(got, want, rtol=1e-12, atol=1e-9)


# -------------------------------------------------------------- retention
def test_zigzag_gather_follows_jpeg_order():
    jpeg = load_matrix("zigzag8_jpeg.txt").ravel()
    b = np.arange(64, dtype=np.int64).reshape(1, 1, 8, 8)
    assert np.array_equal(P.zigzag_gather(b, 64)[0, 0], jpeg)
    kept = P.zigzag_gather(b, 10)
    assert np.array_equal(P.zigzag_scatter(kept, 8), P.retain(b, 10))


def test_zigzag_mask_counts():
    for n in (8, 16, 32):
        for r in (0, 1, 6, 10, n * n // 2, n * n):
            assert P.zigzag_mask(n, r).sum() == r


# -------------------------------------------------------------- inverse
@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_full_retention_reconstructs_exactly(kind, n):
    for img in (random_u8(2 * n, n, 5), np.zeros((n, n), np.uint8),
                np.full((n, n), 255, np.uint8),
                (np.indices((n, n)).sum(0) % 2 * 255).astype(np.uint8)):
        out = P.compress(img, kind, n, n * n)
        assert np.array_equal(out["recon"], img)
        assert out["sse"] == 0 and out["psnr"] == math.inf
    res = random_i16(n, 2 * n, 6)
    res[0, 0], res[0, 1] = 255, -255
    assert np.array_equal(P.compress(res, kind, n, n * n)["recon"], res)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_dc_only_reconstructs_rounded_block_mean(kind, n):
    img = random_u8(2 * n, 2 * n, 7)
    out = P.compress(img, kind, n, 1)
    for by in range(2):
        for bx in range(2):
            blk = img[by * n:(by + 1) * n, bx * n:(bx + 1) * n].astype(np.int64) - 128
            mean = Fraction(int(blk.sum()), n * n)
            want = M.paper_round(mean) + 128        # exact: round() of a rational
            if abs(mean - int(mean)) == Fraction(1, 2):
                want = int(math.copysign(abs(mean) + Fraction(1, 2), mean)) + 128
            assert np.all(out["recon"][by * n:(by + 1) * n, bx * n:(bx + 1) * n] == want)
            assert out["kept"][by, bx, 0] == blk.sum()


def test_round_half_away_div_matches_fraction_rounding():
    for p in range(-600, 601):
        for q in (1, 2, 4, 64, 256, 3):
            x = Fraction(p, q)
            want = (1 if x > 0 else -1) * math.floor(abs(x) + Fraction(1, 2)) if x else 0
            assert P.round_half_away_div(np.array([p]), q)[0] == want


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n,r", [(8, 6), (8, 10), (8, 45), (16, 28), (32, 100)])
def test_inverse_brute_force_rationals(kind, n, r):
    # reconstruct one tile with the exact rational inverse T^-1 B T^-T (no U)
    img = random_u8(n, n, 8)
    out = P.compress(img, kind, n, r)
    b = P.retain(P.forward2d(img, kind, n), r)[0, 0]
    tinv = M.fraction_inverse(M.transform_matrix(kind, n).tolist())
    bb = [[Fraction(int(v)) for v in row] for row in b]
    left = [[sum(tinv[i][k] * bb[k][j] for k in range(n)) for j in range(n)] for i in range(n)]
    x = [[sum(left[i][k] * tinv[j][k] for k in range(n)) for j in range(n)] for i in range(n)]
    for i in range(n):
        for j in range(n):
            v = x[i][j]
            y = (1 if v > 0 else -1) * math.floor(abs(v) + Fraction(1, 2)) if v else 0
            assert out["recon"][i, j] == min(255, max(0, y + 128))


def test_int16_saturation():
    res = np.zeros((8, 8), np.int16)
    b = np.zeros((1, 1, 8, 8), np.int64)
    b[0, 0, 0, 0] = 64 * 40000
    rec = P.inverse2d(b, M.ROUND, 8, np.int16)
    assert np.all(rec == 32767)
    assert P.inverse2d(-b, M.ROUND, 8, np.int16).min() == -32768
    del res


# -------------------------------------------------------------- quantiser
@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
@pytest.mark.parametrize("qstep", (1, 8, 13, 64, 4096))
def test_quantiser_is_uniform_quantiser_of_orthonormal_coefficient(kind, n, qstep):
    # level = round(c / Q) with c = s_v s_u b, except where c / Q lies within the
    # fixed-point multiplier's own rounding error (|c/Q| * 0.5 / MQ) of a tie
    r = rng(9)
    b = r.integers(-262144, 262145, size=(4, n, n)).astype(np.int64)
    mq, dq = P.quant_tables(kind, n, qstep)
    lev = P.quantise(b, mq)
    s = M.scale_vector(kind, n)
    c = np.outer(s, s) * b / qstep
    want = P.round_half_away_float(c)
    window = np.abs(c) * 0.5 / mq + 1e-9
    near_tie = np.abs(np.abs(c) - np.floor(np.abs(c)) - 0.5) < window
    assert near_tie.mean() < 0.2     # most coefficients are checked exactly
    assert np.array_equal(lev[~near_tie], want[~near_tie])
    # dequantised coefficient = 2 * level * Q / (s_v s_u) within half a unit
    deq = P.dequantise(lev, dq)
    assert np.all(np.abs(deq - 2.0 * lev * qstep / np.outer(s, s)) <= 0.5 * np.abs(lev) + 1e-9)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", (16, 32))
def test_quantised_round_trip_error_is_bounded(kind, n):
    # orthonormal reading: per-pixel error stays near the step size on average
    res = synth.laplace_residual(2 * n, 2 * n, seed=10)
    for q in (8, 64):
        out = P.compress(res, kind, n, n * n, qstep=q)
        mse = out["sse"] / res.size
        assert mse < q * q      # far looser than the uniform-noise q^2/12
    out = P.compress(res, kind, n, n * n, qstep=1)
    assert out["sse"] / res.size < 1.0


def test_psnr_closed_forms():
    assert P.psnr(1, 1) == pytest.approx(20 * math.log10(255.0), abs=1e-12)
    assert P.psnr(0, 10) == math.inf
    assert P.psnr(4 * 100, 100) == pytest.approx(20 * math.log10(255.0 / 2.0), abs=1e-12)


# -------------------------------------------------------------- quality
def test_quality_ordering_on_ar1_images():
    # sections 4.1 and 5.2: the round-based approximation is closer to the DCT
    # than the sign-based one and compresses better; the DCT is best
    img = synth.ar1_image(256, 256, rho=0.95, seed=0)
    c = M.dct2_matrix(8)
    a = P.to_tiles(P.level_shift(img), 8).astype(np.float64)
    for r in (6, 10):
        bd = P.retain(c @ a @ c.T, r)
        rec = np.clip(P.round_half_away_float(P.from_tiles(c.T @ bd @ c)) + 128, 0, 255)
        p_dct = P.psnr(P.sse(img, rec.astype(np.uint8)), img.size)
        p_round = P.compress(img, M.ROUND, 8, r)["psnr"]
        p_sign = P.compress(img, M.SIGN, 8, r)["psnr"]
        assert p_dct > p_round > p_sign


def test_paper_literal_form_is_close_to_separable_form():
    img = synth.ar1_image(128, 128, rho=0.95, seed=0)
    for kind in M.KINDS:
        c = M.near_orthogonal(kind, 8)
        cinv = np.linalg.inv(c)
        bl = P.retain(P.forward2d_paper_literal(img, kind, 8), 10)
        rec = np.clip(P.round_half_away_float(P.from_tiles(cinv @ bl @ c)) + 128, 0, 255)
        p_lit = P.psnr(P.sse(img, rec.astype(np.uint8)), img.size)
        assert abs(p_lit - P.compress(img, kind, 8, 10)["psnr"]) < 0.1


# ------------------------------------------------ the exact DCT (section 5)
def _dct_by_cosine_sums(a):
    """c_vu = (2/N) k_v k_u sum_ij a_ij cos((2i+1) v pi / 2N) cos((2j+1) u pi / 2N),
    k_0 = 1/sqrt(2), k = 1 otherwise: the DCT-II written out term by term."""
    n = a.shape[0]
    out = np.zeros((n, n))
    for v in range(n):
        for u in range(n):
            kv = 1 / math.sqrt(2) if v == 0 else 1.0
            ku = 1 / math.sqrt(2) if u == 0 else 1.0
            acc = 0.0
            for i in range(n):
                for j in range(n):
                    acc += a[i, j] * math.cos((2 * i + 1) * v * math.pi / (2 * n)) * \
                        math.cos((2 * j + 1) * u * math.pi / (2 * n))
            out[v, u] = 2.0 / n * kv * ku * acc
    return out


def test_dct_pipeline_against_cosine_sums_and_special_cases():
    rng = np.random.default_rng(21)
    img = rng.integers(0, 256, size=(16, 24), dtype=np.uint8)
    out = P.compress_dct(img, 64)
    # coefficients: the DCT-II written out term by term
    a = img.astype(np.float64) - 128
    for ty in range(2):
        for tx in range(3):
            want = _dct_by_cosine_sums(a[8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8])
            got = out["scaled"][ty, tx]
            want_zz = np.array([want[v, u] for v, u in M.zigzag(8)])
            assert np.allclose(got, want_zz, rtol=0, atol=1e-9)
            # orthonormal: energy is preserved (Parseval)
            assert np.isclose(np.sum(got ** 2), np.sum(a[8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8] ** 2))
    # every coefficient kept: the reconstruction is exact
    assert np.array_equal(out["recon"], img) and out["sse"] == 0 and math.isinf(out["psnr"])
    # r = 1: the block mean, rounded half away from zero (skip blocks whose mean is a tie)
    rec = P.compress_dct(img, 1)["recon"].astype(np.int64)
    for ty in range(2):
        for tx in range(3):
            blk = a[8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8]
            m = blk.mean()
            if abs(abs(m) - math.floor(abs(m)) - 0.5) < 1e-9:
                continue
            want = int(np.sign(m) * math.floor(abs(m) + 0.5)) + 128
            assert np.all(rec[8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8] == want)


def test_dct_pipeline_quality_ordering():
    """Section 5: the exact DCT reconstructs AR(1)-like images better than
    the approximations at every retention level below 64."""
    import synth
    img = synth.ar1_image(64, 64, rho=0.95, seed=2)
    for r in (1, 6, 10, 28, 45):
        dct = P.compress_dct(img, r)["psnr"]
        for kind in M.KINDS:
            assert dct >= P.compress(img, kind, 8, r)["psnr"] - 1e-9
