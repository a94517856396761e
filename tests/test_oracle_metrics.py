"""Pins of the assessment measures against the values the paper prints
(sections 3.1, 4.1, 4.2 and 6.1) and against closed forms."""
import math

import numpy as np
import pytest

from oracle import matrices as M
from oracle import metrics as Q


def sdct8():
    # the signed DCT: sign() of the exact DCT matrix, with S from its T T^T
    t = np.sign(M.dct2_matrix(8)).astype(np.int64)
    s = 1.0 / np.sqrt(np.einsum("ij,ij->i", t, t).astype(np.float64))
    return t, s[:, None] * t


def test_deviation_from_diagonality(paper_values):
    v = paper_values["deviation_from_diagonality"]
    dec = v["decimals"]
    for kind, key in ((M.SIGN, "sign_8"), (M.ROUND, "round_8")):
        t = M.transform_matrix(kind, 8)
        # printed to 4 decimals (0.0579 is 4/69 truncated, not rounded)
        assert abs(Q.deviation_from_diagonality(t @ t.T) - v[key]) < 10.0 ** -dec
    t, _ = sdct8()
    assert round(Q.deviation_from_diagonality(t @ t.T), 2) == v["sdct_8"]
    # exact rational values behind the printed decimals
    assert Q.deviation_from_diagonality(M.transform_matrix(M.SIGN, 8).dot(
        M.transform_matrix(M.SIGN, 8).T)) == pytest.approx(1 / 14, abs=1e-15)
    assert Q.deviation_from_diagonality(M.transform_matrix(M.ROUND, 8).dot(
        M.transform_matrix(M.ROUND, 8).T)) == pytest.approx(4 / 69, abs=1e-15)


def test_deviation_closed_forms():
    assert Q.deviation_from_diagonality(np.diag([1.0, 2.0, 3.0])) == 0.0
    assert Q.deviation_from_diagonality(np.ones((2, 2))) == pytest.approx(0.5)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", (16, 32, 64))
def test_jam_keeps_deviation(kind, n):
    # the JAM recursion keeps delta: it maps T T^T to a direct sum of copies
    t8 = M.transform_matrix(kind, 8)
    t = M.transform_matrix(kind, n)
    assert Q.deviation_from_diagonality(t @ t.T) == pytest.approx(
        Q.deviation_from_diagonality(t8 @ t8.T), abs=1e-12)


def test_total_error_energy_table1(paper_values):
    v = paper_values["total_error_energy"]
    c = M.dct2_matrix(8)
    assert round(Q.total_error_energy(c, M.near_orthogonal(M.ROUND, 8)), 2) == v["round_8"]
    assert round(Q.total_error_energy(c, M.near_orthogonal(M.SIGN, 8)), 2) == v["sign_8"]
    assert round(Q.total_error_energy(c, sdct8()[1]), 2) == v["sdct_8"]
    assert Q.total_error_energy(c, c) == 0.0


def test_coding_gain_klt_and_dct(paper_values):
    v = paper_values["coding_gain"]
    n, rho, dec = v["n"], v["rho"], v["decimals"]
    klt = Q.klt_coding_gain(n, rho)
    assert round(klt, dec) == v["klt"]
    # closed form: det R = (1 - rho^2)^(N-1) for the AR(1) covariance
    assert klt == pytest.approx(-10.0 * (n - 1) / n * math.log10(1 - rho * rho), abs=1e-12)
    for basis in ("rows", "cols"):
        dct = Q.coding_gain(M.dct2_matrix(n), rho, basis)
        assert round(dct, dec) == v["dct"]
        assert round(dct - klt, dec) == v["dct_minus_klt"]


def test_coding_gain_special_cases():
    # identity transform has zero coding gain; KLT eigenbasis attains the KLT gain
    for rho in (0.0, 0.5, 0.95):
        assert Q.coding_gain(np.eye(8), rho) == pytest.approx(0.0, abs=1e-12)
        w, v = np.linalg.eigh(Q.ar1_covariance(8, rho))
        assert Q.coding_gain(v.T, rho) == pytest.approx(Q.klt_coding_gain(8, rho), abs=1e-10)
    # uncorrelated input: every orthonormal transform has zero gain
    assert Q.coding_gain(M.dct2_matrix(8), 0.0) == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("kind", M.KINDS)
def test_coding_gain_below_klt(kind):
    for rho in (0.5, 0.8, 0.95):
        for basis in ("rows", "cols"):
            c = M.near_orthogonal(kind, 8)
            assert Q.coding_gain(c, rho, basis) < Q.klt_coding_gain(8, rho)


def test_additions_table2(paper_values):
    v = paper_values["additions"]
    assert Q.additions_of_chain(M.stage_matrices(M.ROUND)) == v["round_8"]
    assert Q.additions_of_chain(M.stage_matrices(M.SIGN)) == v["sign_8"]


def jam_additions(kind, n):
    # the recursion T_N = M_per diag(T_{N/2}, T_{N/2}) M_add costs two half-size
    # transforms plus the additions of M_add (M_per is a permutation)
    if n == 8:
        return Q.additions_of_chain(M.stage_matrices(kind))
    return (2 * jam_additions(kind, n // 2) + Q.additions_of_factor(M.m_add(n))
            + Q.additions_of_factor(M.m_per(n)))


def test_additions_table4(paper_values):
    v = paper_values["additions"]
    for n in (16, 32):
        assert jam_additions(M.ROUND, n) == v[f"round_{n}"]
        assert jam_additions(M.SIGN, n) == v[f"sign_{n}"]
    # M_add costs exactly N additions and M_per none (section 6)
    for n in (16, 32):
        assert Q.additions_of_factor(M.m_add(n)) == n
        assert Q.additions_of_factor(M.m_per(n)) == 0


def test_additions_of_factor_counts():
    assert Q.additions_of_factor(np.eye(4)) == 0
    assert Q.additions_of_factor(-np.eye(4)) == 0
    assert Q.additions_of_factor(np.array([[1, 1, 1], [0, 2, -1], [0, 0, 0]])) == 3
