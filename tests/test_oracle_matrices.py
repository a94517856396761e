"""Pins of the oracle's transform matrices against what the paper prints and
against closed forms (sections 2, 3, 3.1, 6.1)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft

from conftest import load_matrix
from oracle import matrices as M


def frac_matrix(m):
    return [[Fraction(int(v)) for v in row] for row in np.asarray(m)]


def frac_matmul(a, b):
    n, k, m = len(a), len(b), len(b[0])
    return [[sum(a[i][t] * b[t][j] for t in range(k)) for j in range(m)] for i in range(n)]


# ------------------------------------------------------------------ section 2
def test_dct2_matches_library_and_is_orthonormal():
    for n in (4, 8, 16, 32):
        c = M.dct2_matrix(n)
        lib = scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0)
        assert np.allclose(c, lib, atol=1e-14)
        assert np.allclose(c @ c.T, np.eye(n), atol=1e-13)


def test_dct4_matches_library():
    for n in (2, 4, 8):
        lib = scipy.fft.dct(np.eye(n), type=4, norm="ortho", axis=0)
        assert np.allclose(M.dct4_matrix(n), lib, atol=1e-14)


def test_chen_dct4_factorization_eq2():
    # Eq. 2 as printed gives sqrt(2) C4^IV Ibar4: the product leaves out the
    # sqrt(2/N) normalisation and a column reversal, both of which eq. 3 takes
    # up (its lower block is Ibar C4^IV Ibar, reached through M1 = diag(I, Ibar Q)).
    alpha, beta, _ = M.exact_parameters()
    prod = (M.Q4(np.float64) @ M.A1(beta, np.float64) @ M.A2(np.float64)
            @ M.A3(alpha, np.float64))
    rev = M.counter_identity(4, np.float64)
    assert np.allclose(prod, np.sqrt(2.0) * M.dct4_matrix(4) @ rev, atol=1e-14)


def test_wang_factorization_eq1():
    # C8 = 1/2 P8 diag(C4^II, Ibar C4^IV Ibar) B8, times sqrt(2) per block
    # normalisation: the blocks are the orthonormal 4-point transforms scaled by
    # sqrt(2) so that the product is orthonormal.
    rev = M.counter_identity(4, np.float64)
    mid = np.zeros((8, 8))
    mid[:4, :4] = M.dct2_matrix(4)
    mid[4:, 4:] = rev @ M.dct4_matrix(4) @ rev
    c8 = 0.5 * M.P8(np.float64) @ (np.sqrt(2.0) * mid) @ M.B8(np.float64)
    assert np.allclose(c8, M.dct2_matrix(8), atol=1e-14)


def test_exact_parameters_give_twice_the_dct():
    # section 3: T_C(alpha, beta, gamma) = 2 C8 for the exact constants
    a, b, g = M.exact_parameters()
    t = M.chen_map(a, b, g, dtype=np.float64)
    assert np.allclose(t, 2.0 * M.dct2_matrix(8), atol=1e-14)


def test_exact_factorization_additions_match_table2(paper_values):
    # Chen's exact 8-point factorization needs 26 additions (section 2, Table 2)
    a, b, g = M.exact_parameters()
    chain = [M.P8(np.float64), M.M1(np.float64), M.M2(b, np.float64),
             M.M3(a, g, np.float64), M.M4(a, np.float64), M.B8(np.float64)]
    from oracle.metrics import additions_of_chain
    assert additions_of_chain(chain) == paper_values["additions"]["exact_chen_8"]


# ------------------------------------------------------------------ section 3
def test_sign_round_functions():
    assert [M.paper_sign(x) for x in (-2.5, 0.0, 0.1)] == [-1, 0, 1]
    assert [M.paper_round(x) for x in (-1.5, -0.5, -0.49, 0.5, 1.49, 2.5)] == [-2, -1, 0, 1, 1, 3]


def test_approximate_parameter_vectors():
    # sign of every constant is 1 (section 3, printed vector of ones)
    assert M.approx_parameters(M.SIGN) == (1, (1, 1, 1, 1), (1, 1))
    # round() of the constants; the printed vector is garbled, this is the one
    # that reproduces the printed M^2, M^3 and T^8
    assert M.approx_parameters(M.ROUND) == (1, (1, 1, 1, 0), (1, 0))


@pytest.mark.parametrize("kind,name", [(M.SIGN, "sign"), (M.ROUND, "round")])
def test_stage_matrices_match_printed(kind, name):
    _, _, m2, m3, m4, _ = M.stage_matrices(kind)
    assert np.array_equal(m2, load_matrix(f"m2_{name}.txt"))
    assert np.array_equal(m3, load_matrix(f"m3_{name}.txt"))
    assert np.array_equal(m4, load_matrix("m4.txt"))


@pytest.mark.parametrize("kind,name", [(M.SIGN, "sign"), (M.ROUND, "round")])
def test_t8_matches_printed(kind, name):
    assert np.array_equal(M.transform_matrix(kind, 8), load_matrix(f"t8_{name}.txt"))


def test_factor_inverses_match_printed():
    pairs = [
        (M.stage_matrices(M.SIGN)[2], load_matrix("m2_sign_inv_x2.txt")),
        (M.stage_matrices(M.ROUND)[2], load_matrix("m2_round_inv_x2.txt")),
        (M.stage_matrices(M.SIGN)[3], M.stage_matrices(M.SIGN)[3]),  # printed as M~3 / 2
        (M.stage_matrices(M.ROUND)[3], load_matrix("m3_round_inv_x2.txt")),
        (M.stage_matrices(M.ROUND)[4], load_matrix("m4_inv_x2.txt")),
    ]
    for fwd, inv_x2 in pairs:
        inv = M.fraction_inverse(fwd.tolist())
        assert inv == [[Fraction(int(v), 2) for v in row] for row in inv_x2]
    # B8^-1 = B8^T / 2, P8^-1 = P8^T, M1^-1 = M1^T
    assert M.fraction_inverse(M.B8().tolist()) == [[Fraction(int(v), 2) for v in row]
                                                   for row in M.B8().T]
    for perm in (M.P8(), M.M1()):
        assert np.array_equal(perm @ perm.T, np.eye(8, dtype=np.int64))


@pytest.mark.parametrize("kind,name", [(M.SIGN, "sign"), (M.ROUND, "round")])
def test_inverse_fast_algorithm_eq6_eq7(kind, name):
    # T^-1 = 1/2 B8^T M4^-1 M3^-1 M2^-1 M1^T P8^T with the printed factor inverses
    p8, m1, m2, m3, m4, b8 = M.stage_matrices(kind)
    half = lambda m: [[Fraction(int(v), 2) for v in row] for row in np.asarray(m)]
    m2i = half(load_matrix(f"m2_{name}_inv_x2.txt"))
    m3i = half(m3) if kind == M.SIGN else half(load_matrix("m3_round_inv_x2.txt"))
    m4i = half(load_matrix("m4_inv_x2.txt"))
    chain = half(b8.T)
    for f in (m4i, m3i, m2i, frac_matrix(m1.T), frac_matrix(p8.T)):
        chain = frac_matmul(chain, f)
    t = frac_matrix(M.transform_matrix(kind, 8))
    eye = [[Fraction(int(i == j)) for j in range(8)] for i in range(8)]
    assert frac_matmul(t, chain) == eye
    # and the oracle's exact inverse is the same matrix
    u = M.scaled_inverse(kind, 8)
    assert chain == [[Fraction(int(v), 8) for v in row] for row in u]


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_scaled_inverse_is_exact(kind, n):
    t = M.transform_matrix(kind, n)
    u = M.scaled_inverse(kind, n)
    assert np.array_equal(t @ u, n * np.eye(n, dtype=np.int64))
    assert np.array_equal(u @ t, n * np.eye(n, dtype=np.int64))
    # N T^-1 has entries {0, +-1} (sign-based) or {0, +-1, +-2} (round-based)
    allowed = {-1, 0, 1} if kind == M.SIGN else {-2, -1, 0, 1, 2}
    assert set(np.unique(u).tolist()) <= allowed
    # N is the smallest integer that clears every denominator of T^-1
    inv = M.fraction_inverse(t.tolist())
    assert max(v.denominator for row in inv for v in row) == n


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_entries_and_row_sums(kind, n):
    t = M.transform_matrix(kind, n)
    assert set(np.unique(t).tolist()) <= {-2, -1, 0, 1, 2}
    assert np.all(t[0] == 1)                    # DC row is all ones
    assert np.all(t[1:].sum(axis=1) == 0)       # every AC row sums to zero
    u = M.scaled_inverse(kind, n)
    assert np.all(u[:, 0] == 1)                 # inverse DC column is all ones


# ------------------------------------------------------------------ section 3.1
def test_scale_matrices_match_printed():
    printed = load_matrix("s8_diag_inv_sq.txt")
    assert np.array_equal(M.diag_ttt(M.SIGN, 8), printed[0])
    assert np.array_equal(M.diag_ttt(M.ROUND, 8), printed[1])
    assert np.allclose(M.scale_vector(M.ROUND, 8),
                       [1 / np.sqrt(8), 1 / np.sqrt(6), 0.5, 1 / np.sqrt(12),
                        1 / np.sqrt(8), 1 / np.sqrt(12), 0.5, 1 / np.sqrt(6)], rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind", M.KINDS)
def test_ttt_is_not_diagonal(kind):
    # section 3.1: neither approximation satisfies T T^T = D
    t = M.transform_matrix(kind, 8)
    g = t @ t.T
    assert np.count_nonzero(g - np.diag(np.diag(g))) > 0


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_near_orthogonal_has_unit_rows(kind, n):
    c = M.near_orthogonal(kind, n)
    assert np.allclose(np.einsum("ij,ij->i", c, c), 1.0, atol=1e-14)


# ------------------------------------------------------------------ section 6
def test_m_per_literal_block_reading_is_the_interleave():
    # P_{N-1,N/2}: identity interlaced with zero rows; M_per read as the column
    # blocks [P; 0_{1,N/2}] | [0_{1,N/2}; P]
    for n in (16, 32, 64):
        h = n // 2
        p = np.zeros((n - 1, h), dtype=np.int64)
        for k in range(h):
            p[2 * k, k] = 1
        left = np.vstack([p, np.zeros((1, h), dtype=np.int64)])
        right = np.vstack([np.zeros((1, h), dtype=np.int64), p])
        assert np.array_equal(np.hstack([left, right]), M.m_per(n))


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", (16, 32, 64))
def test_jam_recursion_equals_factorized_form(kind, n):
    p, m1, m2, m3, m4, b = M.jam_factors(kind, n)
    assert np.array_equal(p @ m1 @ m2 @ m3 @ m4 @ b, M.transform_matrix(kind, n))


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", (16, 32, 64))
def test_jam_inverse_factorization(kind, n):
    # T_N^-1 = (4/N) Bcheck^T M4^-1 M3^-1 M2^-1 M1^T Pcheck^T (section 6.1)
    p, m1, m2, m3, m4, b = M.jam_factors(kind, n)
    inv = lambda m: np.array(M.fraction_inverse(m.tolist()), dtype=object)
    chain = (np.array(frac_matrix(b.T), dtype=object) @ inv(m4) @ inv(m3) @ inv(m2)
             @ np.array(frac_matrix(m1.T), dtype=object)
             @ np.array(frac_matrix(p.T), dtype=object)) * Fraction(4, n)
    u = M.scaled_inverse(kind, n)
    assert np.all(chain * n == u)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", (16, 32, 64))
def test_jam_even_rows_mirror_half_transform(kind, n):
    t = M.transform_matrix(kind, n)
    half = M.transform_matrix(kind, n // 2)
    rev = M.counter_identity(n // 2)
    for k in range(n // 2):
        assert np.array_equal(t[2 * k], np.concatenate([half[k], half[k] @ rev]))


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", (16, 32, 64))
def test_jam_odd_rows_act_on_the_difference_vector(kind, n):
    # odd rows apply T_{N/2} to w = Ibar x_top - x_bottom
    t = M.transform_matrix(kind, n)
    half = M.transform_matrix(kind, n // 2)
    rev = M.counter_identity(n // 2)
    for k in range(n // 2):
        assert np.array_equal(t[2 * k + 1], np.concatenate([half[k] @ rev, -half[k]]))


# ------------------------------------------------------------------ zig-zag
def test_zigzag_matches_jpeg_scan():
    jpeg = load_matrix("zigzag8_jpeg.txt").ravel()
    assert [v * 8 + u for v, u in M.zigzag(8)] == jpeg.tolist()


@pytest.mark.parametrize("n", (8, 16, 32, 64))
def test_zigzag_is_a_permutation_by_antidiagonals(n):
    zz = M.zigzag(n)
    assert sorted(zz) == [(v, u) for v in range(n) for u in range(n)]
    d = [v + u for v, u in zz]
    assert d == sorted(d)
    # the scan alternates direction: consecutive cells on a diagonal are adjacent
    for (v0, u0), (v1, u1) in zip(zz, zz[1:]):
        if v0 + u0 == v1 + u1:
            assert abs(v1 - v0) == 1 and abs(u1 - u0) == 1


@pytest.mark.parametrize("n", (8, 16, 32, 64))
def test_zigzag_prefix_keeps_a_prefix_of_every_column(n):
    # for every r, the rows kept in column u by the first r scan positions are
    # 0 .. c_u - 1 (the JAM kernels mask each column by such a count)
    pos = {vu: k for k, vu in enumerate(M.zigzag(n))}
    for r in range(n * n + 1):
        for u in range(n):
            kept = [v for v in range(n) if pos[(v, u)] < r]
            assert kept == list(range(len(kept)))


# --------------------------------------- comparison transforms of section 4
def test_comparison_kinds_are_the_section4_matrices(paper_values):
    """transform_matrix serves the 8-point comparison transforms: their
    orthonormalised forms reproduce the total error energies of Table 1
    (WHT 5.05, HT 47.61, SDCT 3.32) and SDCT's deviation from diagonality."""
    from oracle import metrics as Q
    c = M.dct2_matrix(8)
    want = {M.WHT: 5.05, M.HT: 47.61, M.SDCT: paper_values["total_error_energy"]["sdct_8"]}
    for kind in M.COMPARISON_KINDS:
        assert round(Q.total_error_energy(c, M.near_orthogonal(kind, 8)), 2) == want[kind]
        t = M.transform_matrix(kind, 8)
        # every AC row sums to zero (the level shift folds into the DC term)
        assert np.all(t[1:].sum(axis=1) == 0) and np.all(t[0] == 1)
        # the exact inverse is integral after scaling by 8
        u = M.scaled_inverse(kind, 8)
        assert np.array_equal(t @ u, 8 * np.eye(8, dtype=np.int64))
    t = M.transform_matrix(M.SDCT, 8)
    assert np.array_equal(t, np.sign(M.dct2_matrix(8)).astype(np.int64))
    assert round(Q.deviation_from_diagonality(t @ t.T), 2) == \
        paper_values["deviation_from_diagonality"]["sdct_8"]
    for kind in (M.WHT, M.HT):
        t = M.transform_matrix(kind, 8)
        assert np.array_equal(t @ t.T, 8 * np.eye(8, dtype=np.int64))
    with pytest.raises(ValueError):
        M.transform_matrix(M.WHT, 16)


def test_comparison_kinds_in_the_pipeline():
    """The pipeline's special cases hold for the comparison transforms:
    r = 64 reconstructs exactly, r = 1 gives the rounded block mean."""
    from oracle import pipeline as P
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(16, 24), dtype=np.uint8)
    for kind in M.COMPARISON_KINDS:
        assert np.array_equal(P.compress(img, kind, 8, 64)["recon"], img)
        rec = P.compress(img, kind, 8, 1)["recon"]
        tiles = img.reshape(2, 8, 3, 8).astype(np.int64).sum(axis=(1, 3))
        mean = np.sign(tiles) * ((2 * np.abs(tiles - 0) + 64) // 128)   # round(sum / 64)
        want = np.repeat(np.repeat(mean, 8, axis=0), 8, axis=1)
        assert np.array_equal(rec.astype(np.int64), want)
