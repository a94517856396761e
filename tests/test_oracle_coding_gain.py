"""Pins of the coding-gain measures (section 4.1): the paper's description of
its missing figure (which selects the reading of g_k), the 2D empirical gain
against the AR(1) model's population moments, the variance and moment sums
against brute force, and the paper-literal 2D form against an element-wise
evaluation."""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import matrices as M
from oracle import metrics as Q
from oracle import pipeline as P
import synth

RHOS = [0.05 * i for i in range(1, 20)] + [0.97, 0.99, 0.999]


def orthonormal(t):
    t = np.asarray(t, dtype=np.float64)
    return t / np.sqrt(np.einsum("ij,ij->i", t, t))[:, None]


def rel_gain(c, rho, basis):
    return Q.coding_gain(c, rho, basis) - Q.klt_coding_gain(c.shape[0], rho)


def test_comparison_transforms_match_table1(paper_values):
    # total error energies of Table 1 pin the row orders of WHT and HT
    c = M.dct2_matrix(8)
    wht = orthonormal(M.hadamard_matrix(8, "sequency"))
    ht = orthonormal(M.hadamard_matrix(8, "natural"))
    assert round(Q.total_error_energy(c, wht), 2) == 5.05
    assert round(Q.total_error_energy(c, ht), 2) == 47.61
    assert round(Q.total_error_energy(c, orthonormal(M.sdct_matrix(8))), 2) == \
        paper_values["total_error_energy"]["sdct_8"]
    # Sylvester's matrix is orthogonal: H H^T = n I
    for n in (8, 16, 32):
        h = M.hadamard_matrix(n)
        assert np.array_equal(h @ h.T, n * np.eye(n, dtype=np.int64))


def test_figure2_description_selects_the_columns_reading():
    # section 4.1 describes its figure: the DCT is closest to the KLT,
    # followed by HT and WHT (equal values); the proposed transforms beat the
    # SDCT; as rho -> 1 the round-based approximation performs as well as
    # HT and WHT.  With g_k the columns of C^-1 all of it holds; with rows
    # the round-based transform overtakes WHT.
    dct = M.dct2_matrix(8)
    wht = orthonormal(M.hadamard_matrix(8, "sequency"))
    ht = orthonormal(M.hadamard_matrix(8, "natural"))
    sdct = orthonormal(M.sdct_matrix(8))
    c_round = M.near_orthogonal(M.ROUND, 8)
    c_sign = M.near_orthogonal(M.SIGN, 8)
    for rho in RHOS:
        g = {name: rel_gain(c, rho, "cols") for name, c in
             (("dct", dct), ("wht", wht), ("ht", ht), ("round", c_round), ("sign", c_sign),
              ("sdct", sdct))}
        assert g["wht"] == pytest.approx(g["ht"], abs=1e-12)
        assert g["dct"] > g["wht"] > g["round"] > g["sign"], rho
        assert g["round"] > g["sdct"] and g["sign"] > g["sdct"], rho
    near_one = 1.0 - 1e-7
    assert abs(rel_gain(c_round, near_one, "cols") - rel_gain(wht, near_one, "cols")) < 2e-3
    # the literal reading contradicts the description: above rho ~ 0.95 the
    # round-based transform would beat WHT, by 0.06 dB in the limit
    assert rel_gain(c_round, near_one, "rows") - rel_gain(wht, near_one, "rows") > 0.05
    assert rel_gain(c_round, 0.9, "rows") < rel_gain(wht, 0.9, "rows")


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
@pytest.mark.parametrize("basis", ("rows", "cols"))
def test_2d_gain_of_population_moments_is_twice_the_1d_gain(kind, n, basis):
    # separable AR(1) field: coefficient (v, u) of C A C^T has variance
    # (C R C^T)_vv (C R C^T)_uu, the pixels have unit variance
    c = M.near_orthogonal(kind, n)
    for rho in (0.3, 0.9, 0.95):
        d = np.diag(c @ Q.ar1_covariance(n, rho) @ c.T)
        g2 = Q.coding_gain_2d(c, np.outer(d, d), 1.0, basis)
        assert g2 == pytest.approx(2 * Q.coding_gain(c, rho, basis), rel=1e-12, abs=1e-12)
        # scaling the field leaves the gain unchanged
        assert Q.coding_gain_2d(c, 9.0 * np.outer(d, d), 9.0, basis) == pytest.approx(g2, rel=1e-12)


def test_2d_gain_of_white_noise_under_the_dct_is_zero():
    c = M.dct2_matrix(8)
    assert Q.coding_gain_2d(c, np.full((8, 8), 3.0), 3.0, "cols") == pytest.approx(0.0, abs=1e-12)
    assert Q.coding_gain_2d(c, np.full((8, 8), 3.0), 0.0, "cols") != Q.coding_gain_2d(
        c, np.full((8, 8), 3.0), 0.0, "cols")   # NaN for a constant image
    v = np.full((8, 8), 3.0)
    v[2, 5] = 0.0
    assert Q.coding_gain_2d(c, v, 3.0, "cols") == math.inf


def test_variance_from_sums_brute_force():
    r = np.random.default_rng(3)
    for _ in range(20):
        x = r.integers(-40000, 40000, size=int(r.integers(1, 300)))
        s1, s2 = int(x.sum()), int((x.astype(object) ** 2).sum())
        want = Fraction(sum(int(v) ** 2 for v in x), len(x)) - Fraction(int(x.sum()), len(x)) ** 2
        assert Q.variance_from_sums(len(x), s1, s2) == float(want)
        assert Q.variance_from_sums(len(x), s1, s2) == pytest.approx(float(np.var(x)), rel=1e-12)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", (8, 16))
def test_coefficient_moments_brute_force(kind, n):
    # every coefficient by its defining double sum, tile by tile
    img = synth.ar1_image(2 * n, 3 * n, rho=0.9, seed=5)
    t = M.transform_matrix(kind, n).tolist()
    a = img.astype(np.int64) - 128
    s1 = [[0] * n for _ in range(n)]
    s2 = [[0] * n for _ in range(n)]
    for by in range(2):
        for bx in range(3):
            blk = a[by * n:(by + 1) * n, bx * n:(bx + 1) * n].tolist()
            for v in range(n):
                for u in range(n):
                    b = sum(t[v][i] * blk[i][j] * t[u][j] for i in range(n) for j in range(n))
                    s1[v][u] += b
                    s2[v][u] += b * b
    mom = P.coefficient_moments(img, kind, n)
    assert mom["tiles"] == 6 and mom["pixels"] == img.size
    assert mom["s1"].tolist() == s1 and mom["s2"].tolist() == s2
    assert mom["a1"] == int(a.sum()) and mom["a2"] == int((a * a).sum())
    # int16 input is not level-shifted
    r16 = synth.laplace_residual(n, n, seed=1)
    assert P.coefficient_moments(r16, kind, n)["a1"] == int(r16.astype(np.int64).sum())


@pytest.mark.parametrize("kind", M.KINDS)
def test_empirical_gain_approaches_the_model(kind):
    # a large unclipped AR(1) field with a short correlation length: the
    # measured 2D gain approaches twice the model's 1D gain
    rho = 0.5
    y = synth.ar1_field(1024, 1024, rho, synth.rng_for(11))
    img = np.round(1000.0 * y).astype(np.int16)
    c = M.near_orthogonal(kind, 8)
    for basis in ("rows", "cols"):
        got = P.empirical_coding_gain(img, kind, 8, basis)
        assert got == pytest.approx(2 * Q.coding_gain(c, rho, basis), abs=0.02)


@pytest.mark.parametrize("kind", M.KINDS)
def test_paper_literal_form_elementwise(kind):
    # B = C A C^-1 evaluated entry by entry, with C^-1 = (U / N) S'^-1 from the
    # exact integer inverse U = N T^-1 (so no floating-point matrix inverse is
    # shared with the function under test)
    img = synth.ar1_image(16, 24, rho=0.9, seed=2)
    n = 8
    s = M.scale_vector(kind, n)
    t = M.transform_matrix(kind, n)
    u = M.scaled_inverse(kind, n)
    c = s[:, None] * t
    cinv = (u / n) / s[None, :]
    got = P.forward2d_paper_literal(img, kind, n)
    a = img.astype(np.int64) - 128
    for by in range(2):
        for bx in range(3):
            blk = a[by * n:(by + 1) * n, bx * n:(bx + 1) * n]
            for v in range(n):
                for w in range(n):
                    want = sum(c[v, i] * blk[i, j] * cinv[j, w]
                               for i in range(n) for j in range(n))
                    assert got[by, bx, v, w] == pytest.approx(want, abs=1e-9)
    # and C^-1 is not C^T for these transforms (the two 2D forms differ)
    assert not np.allclose(cinv, c.T)
