"""Transform matrices of the paper, built exactly from their definitions.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline may use this module.  It shares no code with the HIP library.

Everything here is dense and exact: integer matrices are numpy int64, inverses
are computed with Python ``Fraction`` Gauss-Jordan elimination, and the
floating-point objects (exact DCT, scale factors) are float64.

Sources in the paper:
  * section 2: DCT-II/DCT-IV definitions, counter-identity, Wang's
    factorization (eq. 1, P8, B8), Chen's DCT-IV factorization (eq. 2:
    Q, A1, A2, A3) and the 8-point Chen factorization (eq. 3: M1..M4, P4, B4,
    C-tilde);
  * section 3: the parametric map T_C(alpha, beta, gamma), the sign and
    round functions, the approximated parameter vectors, T~8 (eq. 4) and
    T^8 (eq. 5), the inverse factorizations (eqs. 6, 7);
  * section 3.1: S' = sqrt(diag(T T^T))^-1 and the near-orthogonal C = S T;
  * section 6 and 6.1: the Jridi-Alfalou-Meher recursion (M_add, M_per) and
    the Chen-JAM transforms for N = 16, 32 with their factorizations.

Readings (the paper is garbled or silent here):
  * The round() parameter vector printed in section 3 does not reproduce the
    printed M^2, T^8 or S^8.  The vector is therefore computed by applying the
    paper's round() to the exact parameters, which gives alpha=1,
    beta=(1,1,1,0), gamma=(1,0) and reproduces every printed matrix.
  * The block layout printed for M_per is dimensionally inconsistent; it is
    read as the interleave (output 2k <- top half k, output 2k+1 <- bottom
    half k), which is what a column-block reading of the printed blocks
    gives.
  * The JAM recursion proposed in section 6.1 drops the 1/sqrt(2) factor of
    the generic JAM form; S_N absorbs the scale.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
import math

import numpy as np

# transform ids used throughout: 1 = sign-based T~ (eq. 4), 2 = round-based T^ (eq. 5);
# 8-point comparison transforms of section 4: 3 = WHT (sequency order),
# 4 = SDCT (sign of the DCT matrix), 5 = HT (Sylvester's natural order)
SIGN = 1
ROUND = 2
WHT = 3
SDCT = 4
HT = 5
KINDS = (SIGN, ROUND)
COMPARISON_KINDS = (WHT, SDCT, HT)
SIZES = (8, 16, 32, 64)   # block lengths: the recursion of section 6.1 to its 64-point level


# ---------------------------------------------------------------- section 2
def dct2_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II, [C]_{m,k} = sqrt(2/N) c_m cos(m(2k+1)pi/(2N)).
    Section 2: the DCT-II."""
    m = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    c = np.where(m == 0, 1.0 / math.sqrt(2.0), 1.0)
    return math.sqrt(2.0 / n) * c * np.cos(m * (2 * k + 1) * math.pi / (2 * n))


def dct4_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-IV, [C]_{m,k} = sqrt(2/N) cos((2m+1)(2k+1)pi/(4N)).
    Section 2: the DCT-IV of the factorization in eq. 2."""
    m = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    return math.sqrt(2.0 / n) * np.cos((2 * m + 1) * (2 * k + 1) * math.pi / (4 * n))


def counter_identity(n: int, dtype=np.int64) -> np.ndarray:
    """Ibar_n: ones on the anti-diagonal.  Section 2: the counter-identity."""
    return np.fliplr(np.eye(n, dtype=dtype))


def _blockdiag(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Direct sum of two blocks (the block-diagonal factors of section 2)."""
    dt = np.result_type(a, b)
    out = np.zeros((a.shape[0] + b.shape[0], a.shape[1] + b.shape[1]), dtype=dt)
    out[: a.shape[0], : a.shape[1]] = a
    out[a.shape[0]:, a.shape[1]:] = b
    return out


def _butterfly(n: int, dtype=np.int64) -> np.ndarray:
    """[[I, Ibar], [Ibar, -I]] of order n (B8, B4 and M_add share this form).
    Section 2 (B8 of eq. 1, B4 of eq. 3) and section 6.1 (M_add)."""
    h = n // 2
    eye = np.eye(h, dtype=dtype)
    rev = counter_identity(h, dtype)
    return np.block([[eye, rev], [rev, -eye]])


def P8(dtype=np.int64) -> np.ndarray:
    """Output permutation of eq. 1: row i selects input column perm[i]."""
    perm = [0, 7, 1, 6, 2, 5, 3, 4]
    m = np.zeros((8, 8), dtype=dtype)
    for i, j in enumerate(perm):
        m[i, j] = 1
    return m


def B8(dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 1: the butterfly B8."""
    return _butterfly(8, dtype)


def P4(dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 3: the permutation P4."""
    perm = [0, 3, 1, 2]
    m = np.zeros((4, 4), dtype=dtype)
    for i, j in enumerate(perm):
        m[i, j] = 1
    return m


def B4(dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 3: the butterfly B4."""
    return _butterfly(4, dtype)


def Q4(dtype=np.int64) -> np.ndarray:
    """Q of eq. 2 (swaps entries 1 and 2)."""
    perm = [0, 2, 1, 3]
    m = np.zeros((4, 4), dtype=dtype)
    for i, j in enumerate(perm):
        m[i, j] = 1
    return m


def A1(beta, dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 2: the factor A1, with the parameters beta of section 3."""
    b0, b1, b2, b3 = beta
    return np.array([[b0, 0, 0, b3],
                     [0, b2, b1, 0],
                     [0, b1, -b2, 0],
                     [b3, 0, 0, -b0]], dtype=dtype)


def A2(dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 2: the factor A2."""
    return np.array([[1, 1, 0, 0],
                     [1, -1, 0, 0],
                     [0, 0, -1, 1],
                     [0, 0, 1, 1]], dtype=dtype)


def A3(alpha, dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 2: the factor A3, with the parameter alpha of section 3."""
    a = alpha
    return np.array([[0, 0, 0, 1],
                     [0, a, a, 0],
                     [0, -a, a, 0],
                     [1, 0, 0, 0]], dtype=dtype)


def Ctilde(alpha, gamma, dtype=np.int64) -> np.ndarray:
    """diag(C2^II, Ibar C2^IV Ibar) in Chen's parametrisation (eq. 3)."""
    a = alpha
    g0, g1 = gamma
    return np.array([[a, a, 0, 0],
                     [a, -a, 0, 0],
                     [0, 0, -g0, g1],
                     [0, 0, g1, g0]], dtype=dtype)


def M1(dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 3: the stage M1."""
    return _blockdiag(np.eye(4, dtype=dtype), counter_identity(4, dtype) @ Q4(dtype))


def M2(beta, dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 3: the stage M2 with the parameters beta (section 3)."""
    return _blockdiag(P4(dtype), A1(beta, dtype))


def M3(alpha, gamma, dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 3: the stage M3 with the parameters alpha, gamma (section 3)."""
    return _blockdiag(Ctilde(alpha, gamma, dtype), A2(dtype))


def M4(alpha, dtype=np.int64) -> np.ndarray:
    """Section 2, eq. 3: the stage M4 with the parameter alpha (section 3)."""
    return _blockdiag(B4(dtype), A3(alpha, dtype))


def chen_map(alpha, beta, gamma, dtype=np.int64) -> np.ndarray:
    """T_C(alpha, beta, gamma) = P8 M1 M2(beta) M3(alpha, gamma) M4(alpha) B8.
    Section 3: the parametric map of the factorization in eq. 3."""
    return (P8(dtype) @ M1(dtype) @ M2(beta, dtype) @ M3(alpha, gamma, dtype)
            @ M4(alpha, dtype) @ B8(dtype))


# ---------------------------------------------------------------- section 3
def exact_parameters():
    """The constants of Chen's factorization (section 3, exact values)."""
    alpha = math.cos(math.pi / 4)
    beta = tuple(math.cos((2 * n + 1) * math.pi / 16) for n in range(4))
    gamma = tuple(math.cos((2 * n + 1) * math.pi / 8) for n in range(2))
    return alpha, beta, gamma


def paper_sign(x: float) -> int:
    """Section 3: the sign() function."""
    return 1 if x > 0 else (-1 if x < 0 else 0)


def paper_round(x: float) -> int:
    """round(x) = sign(x) * floor(|x| + 1/2)  (section 3)."""
    return paper_sign(x) * math.floor(abs(x) + 0.5)


def approx_parameters(kind: int):
    """(alpha, beta, gamma) after applying sign() (kind 1) or round() (kind 2).
    Section 3: the approximated parameter vectors (round: see the module docstring)."""
    f = paper_sign if kind == SIGN else paper_round
    alpha, beta, gamma = exact_parameters()
    return f(alpha), tuple(f(b) for b in beta), tuple(f(g) for g in gamma)


def stage_matrices(kind: int):
    """The integer factors (P8, M1, M2, M3, M4, B8) of eq. 4 / eq. 5."""
    a, b, g = approx_parameters(kind)
    return P8(), M1(), M2(b), M3(a, g), M4(a), B8()


@lru_cache(maxsize=None)
def _t8(kind: int) -> np.ndarray:
    """Section 3, eqs. 4 and 5: the sign-based and round-based 8-point approximations."""
    a, b, g = approx_parameters(kind)
    t = chen_map(a, b, g)
    t.setflags(write=False)
    return t


# ---------------------------------------------------------------- section 6
def m_add(n: int, dtype=np.int64) -> np.ndarray:
    """M_add_N = [[I, Ibar], [Ibar, -I]] (N additions).
    Section 6.1: M_add of the JAM recursion."""
    return _butterfly(n, dtype)


def m_per(n: int, dtype=np.int64) -> np.ndarray:
    """M_per_N: output 2k takes input k, output 2k+1 takes input N/2 + k.
    Section 6.1: M_per of the JAM recursion (read as the interleave)."""
    m = np.zeros((n, n), dtype=dtype)
    h = n // 2
    for k in range(h):
        m[2 * k, k] = 1
        m[2 * k + 1, h + k] = 1
    return m


@lru_cache(maxsize=None)
def transform_matrix(kind: int, n: int) -> np.ndarray:
    """T_N of the paper as an int64 matrix (read-only).

    N = 8: eq. 4 (kind 1) or eq. 5 (kind 2).  N > 8: the recursion of
    section 6.1, T_N = M_per_N diag(T_{N/2}, T_{N/2}) M_add_N.
    The comparison transforms of section 4 (kinds 3, 4, 5) are 8-point
    matrices: the Hadamard matrix in sequency order (WHT) or natural order
    (HT) and the signed DCT.
    """
    if kind in COMPARISON_KINDS:
        if n != 8:
            raise ValueError("the comparison transforms are 8-point transforms")
        t = (sdct_matrix(8) if kind == SDCT else
             hadamard_matrix(8, "sequency" if kind == WHT else "natural"))
        t.setflags(write=False)
        return t
    if kind not in KINDS:
        raise ValueError(f"unknown transform kind {kind}")
    if n == 8:
        return _t8(kind)
    if n < 8 or n & (n - 1):
        raise ValueError(f"N must be a power of two >= 8, got {n}")
    half = transform_matrix(kind, n // 2)
    t = m_per(n) @ _blockdiag(half, half) @ m_add(n)
    t.setflags(write=False)
    return t


def jam_factors(kind: int, n: int):
    """Factors (Pcheck_N, M_N^(1), M_N^(2), M_N^(3), M_N^(4), Bcheck_N) of the
    expanded Chen-JAM factorization (section 6.1).  Their product is T_N."""
    if n == 8:
        return stage_matrices(kind)
    p, m1, m2, m3, m4, b = jam_factors(kind, n // 2)
    return (m_per(n) @ _blockdiag(p, p), _blockdiag(m1, m1), _blockdiag(m2, m2),
            _blockdiag(m3, m3), _blockdiag(m4, m4), _blockdiag(b, b) @ m_add(n))


# ---------------------------------------------------------- exact inverses
def fraction_inverse(m) -> list:
    """Exact inverse of a square integer/rational matrix (Gauss-Jordan on
    Fractions).  Returns a list of lists of Fraction; raises on singular input.
    Exact rational inversion, used for the inverses of sections 3 and 6.1."""
    n = len(m)
    a = [[Fraction(int(m[i][j])) if not isinstance(m[i][j], Fraction) else m[i][j]
          for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for col in range(n):
        piv = next((r for r in range(col, n) if a[r][col] != 0), None)
        if piv is None:
            raise ZeroDivisionError("singular matrix")
        a[col], a[piv] = a[piv], a[col]
        p = a[col][col]
        a[col] = [v / p for v in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [vr - f * vc for vr, vc in zip(a[r], a[col])]
    return [row[n:] for row in a]


@lru_cache(maxsize=None)
def scaled_inverse(kind: int, n: int) -> np.ndarray:
    """U_N = N * T_N^-1 as int64 (read-only).

    Computed by exact rational inversion; raises if N*T_N^-1 is not integral.
    Sections 3 (eqs. 6, 7) and 6.1: the exact inverse, scaled to integers.
    """
    inv = fraction_inverse(transform_matrix(kind, n).tolist())
    u = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        for j in range(n):
            v = inv[i][j] * n
            if v.denominator != 1:
                raise ArithmeticError("N * T^-1 is not integral")
            u[i, j] = v.numerator
    u.setflags(write=False)
    return u


# ------------------------------------------------------------ section 3.1
def diag_ttt(kind: int, n: int) -> np.ndarray:
    """diag(T_N T_N^T) as int64.  Section 3.1: the diagonal of T T^T."""
    t = transform_matrix(kind, n)
    return np.einsum("ij,ij->i", t, t)


def scale_vector(kind: int, n: int) -> np.ndarray:
    """s = diag(S') = 1/sqrt(diag(T T^T)) in float64.
    Section 3.1: the orthogonalising diagonal S'."""
    return 1.0 / np.sqrt(diag_ttt(kind, n).astype(np.float64))


def near_orthogonal(kind: int, n: int) -> np.ndarray:
    """C = S' T (float64).  Section 3.1: the near-orthogonal approximation."""
    return scale_vector(kind, n)[:, None] * transform_matrix(kind, n).astype(np.float64)


# ------------------------------------------- comparison transforms (section 4)
def hadamard_matrix(n: int, order: str = "natural", dtype=np.int64) -> np.ndarray:
    """The n-point Hadamard matrix of Sylvester's construction (entries +-1).

    order="natural": Sylvester's row order, the HT of section 4;
    order="sequency": rows sorted by their number of sign changes, the WHT of
    section 4 (the order that puts low frequencies first, like the DCT).
    Table 1 pins both orders: their total error energies against the 8-point
    DCT are 47.61 (HT) and 5.05 (WHT)."""
    if n < 1 or n & (n - 1):
        raise ValueError("n must be a power of two")
    h = np.ones((1, 1), dtype=dtype)
    while h.shape[0] < n:
        h = np.block([[h, h], [h, -h]])
    if order == "natural":
        return h
    if order == "sequency":
        changes = [int(np.count_nonzero(r[1:] != r[:-1])) for r in h]
        return h[np.argsort(changes, kind="stable")]
    raise ValueError(f"unknown order {order}")


def sdct_matrix(n: int = 8, dtype=np.int64) -> np.ndarray:
    """The signed DCT, sign() of every entry of the exact DCT-II matrix
    (section 4's SDCT; Table 1 gives its total error energy 3.32)."""
    return np.sign(dct2_matrix(n)).astype(dtype)


# ---------------------------------------------------------------- zig-zag
@lru_cache(maxsize=None)
def zigzag(n: int) -> tuple:
    """JPEG zig-zag scan of an n x n block as ((v, u), ...).

    v is the vertical frequency (row), u the horizontal one (column).
    Anti-diagonal d = v + u is visited in increasing order; on odd d the scan
    runs from (0, d) towards increasing v, on even d from (d, 0) towards
    decreasing v; positions outside the square are skipped.
    Section 5.1: the zig-zag order of the retained coefficients.
    """
    order = []
    for d in range(2 * n - 1):
        if d % 2 == 1:
            cells = [(v, d - v) for v in range(0, d + 1)]
        else:
            cells = [(v, d - v) for v in range(d, -1, -1)]
        order.extend((v, u) for v, u in cells if v < n and u < n)
    return tuple(order)
