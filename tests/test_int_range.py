"""Integer range of the fused path: every intermediate fits int32 for every
input the API accepts (uint8, and int16 over its whole range).

Each node of the kernels' butterflies is a linear form of the tile's pixels,
so over |x| <= M its largest magnitude is M times the L1 norm of the form.
The model below runs the node structure of the 8-point factorisation (eqs.
4-7: B8, M4, M3, M2, M1 and P8 forward; their inverses with K8 = 16 T^-1)
and of the Chen-JAM recursion (section 6.1, K_N = 2N T_N^-1) on linear
forms instead of numbers.  The model is first checked against the oracle's
T_N and N T_N^-1, then used to bound every node of the 2D path:
  forward rows, forward columns, inverse columns (zig-zag mask applied or
  dequantised levels), inverse rows."""
import math

import numpy as np
import pytest

from oracle import matrices as M

INT32 = 2 ** 31 - 1
XMAX = 32768                      # largest |int16|


class Forms:
    """Collects the L1 norm of every node created while a butterfly runs."""

    def __init__(self):
        self.peak = 0.0

    def __call__(self, v):
        a = np.abs(v)
        norm = a.reshape(a.shape[0], -1).sum(1).max() if a.ndim > 1 else a.sum()
        self.peak = max(self.peak, float(norm))
        return v


def hadamard8(x, sequency, t):
    y = [t(x[i] + x[i + 4]) for i in range(4)] + [t(x[i] - x[i + 4]) for i in range(4)]
    z = [None] * 8
    for h in range(2):
        for i in range(2):
            z[4 * h + i] = t(y[4 * h + i] + y[4 * h + i + 2])
            z[4 * h + i + 2] = t(y[4 * h + i] - y[4 * h + i + 2])
    nat = [None] * 8
    for q in range(4):
        nat[2 * q] = t(z[2 * q] + z[2 * q + 1])
        nat[2 * q + 1] = t(z[2 * q] - z[2 * q + 1])
    return [nat[i] for i in (0, 4, 6, 2, 3, 7, 5, 1)] if sequency else nat


def hadamard8_inv(X, sequency, t):
    nat = [None] * 8
    if sequency:
        for k, i in enumerate((0, 4, 6, 2, 3, 7, 5, 1)):
            nat[i] = X[k]
    else:
        nat = list(X)
    return [t(2 * v) for v in hadamard8(nat, False, t)]


def sdct8(x, t):
    s = [t(x[i] + x[7 - i]) for i in range(4)]
    d = [t(x[i] - x[7 - i]) for i in range(4)]
    e0, e1, e2, e3 = t(s[0] + s[3]), t(s[1] + s[2]), t(s[0] - s[3]), t(s[1] - s[2])
    a, b, c, p = t(d[0] - d[1]), t(d[2] + d[3]), t(d[2] - d[3]), t(d[0] + d[1])
    return [t(e0 + e1), t(p + b), t(e2 + e3), t(a - b), t(e0 - e1), t(a + b), t(e2 - e3),
            t(a + c)]


def sdct8_inv(X, t):
    f0, f1, f2, f3 = t(X[0] + X[4]), t(X[0] - X[4]), t(X[2] + X[6]), t(X[2] - X[6])
    s = [t(2 * (f0 + f2)), t(2 * (f1 + f3)), t(2 * (f1 - f3)), t(2 * (f0 - f2))]
    d = [t(4 * (X[1] + X[3])), t(4 * (X[1] - X[5])), t(4 * (X[7] - X[3])), t(4 * (X[5] - X[7]))]
    return [t(s[i] + d[i]) for i in range(4)] + [t(s[3 - i] - d[3 - i]) for i in range(4)]


def fwd8(x, kind, t):
    if kind in (M.WHT, M.HT):
        return hadamard8(x, kind == M.WHT, t)
    if kind == M.SDCT:
        return sdct8(x, t)
    y = [t(x[0] + x[7]), t(x[1] + x[6]), t(x[2] + x[5]), t(x[3] + x[4]),
         t(x[3] - x[4]), t(x[2] - x[5]), t(x[1] - x[6]), t(x[0] - x[7])]
    z0, z1, z2, z3 = t(y[0] + y[3]), t(y[1] + y[2]), t(y[1] - y[2]), t(y[0] - y[3])
    z4, z5, z6, z7 = y[7], t(y[5] + y[6]), t(y[6] - y[5]), y[4]
    w0, w1 = t(z0 + z1), t(z0 - z1)
    w2, w3 = (t(z3 - z2), t(z2 + z3)) if kind == M.SIGN else (-z2, z3)
    w4, w5, w6, w7 = t(z4 + z5), t(z4 - z5), t(z7 - z6), t(z6 + z7)
    v4, v7 = (t(w4 + w7), t(w4 - w7)) if kind == M.SIGN else (w4, -w7)
    v5, v6 = t(w5 + w6), t(w5 - w6)
    return [w0, v4, w3, v6, w1, v5, w2, v7]


def inv8(X, kind, t):
    if kind in (M.WHT, M.HT):
        return hadamard8_inv(X, kind == M.WHT, t)
    if kind == M.SDCT:
        return sdct8_inv(X, t)
    v0, v1, v2, v3, v4, v5, v6, v7 = X[0], X[2], X[4], X[6], X[1], X[5], X[3], X[7]
    w0, w1, w2, w3 = t(2 * v0), t(2 * v2), t(2 * v3), t(2 * v1)
    w4, w7 = (t(v4 + v7), t(v4 - v7)) if kind == M.SIGN else (t(2 * v4), t(-2 * v7))
    w5, w6 = t(v5 + v6), t(v5 - v6)
    z0, z1 = t(w0 + w1), t(w0 - w1)
    z2, z3 = (t(w3 - w2), t(w2 + w3)) if kind == M.SIGN else (t(-2 * w2), t(2 * w3))
    z4, z5, z6, z7 = t(w4 + w5), t(w4 - w5), t(w7 - w6), t(w6 + w7)
    y0, y1, y2, y3 = t(z0 + z3), t(z1 + z2), t(z1 - z2), t(z0 - z3)
    y4, y5, y6, y7 = t(2 * z7), t(z5 - z6), t(z5 + z6), t(2 * z4)
    return [t(y0 + y7), t(y1 + y6), t(y2 + y5), t(y3 + y4),
            t(y3 - y4), t(y2 - y5), t(y1 - y6), t(y0 - y7)]


def fwd(x, kind, t):
    n = len(x)
    if n == 8:
        return fwd8(x, kind, t)
    h = n // 2
    u = fwd([t(x[i] + x[n - 1 - i]) for i in range(h)], kind, t)
    w = fwd([t(x[h - 1 - i] - x[h + i]) for i in range(h)], kind, t)
    return [u[k // 2] if k % 2 == 0 else w[k // 2] for k in range(n)]


def inv(X, kind, t):
    n = len(X)
    if n == 8:
        return inv8(X, kind, t)
    h = n // 2
    p = inv([X[2 * k] for k in range(h)], kind, t)
    q = inv([X[2 * k + 1] for k in range(h)], kind, t)
    return [t(p[i] + q[h - 1 - i]) for i in range(h)] + [t(p[h - 1 - i] - q[i]) for i in range(h)]


def unit(n):
    return [np.eye(n)[i] for i in range(n)]


def peak(fn, forms, kind):
    t = Forms()
    fn(forms, kind, t)
    return t.peak


def mask(n, r):
    m = np.zeros((n, n))
    for p in M.zigzag(n)[:r]:
        m[p] = 1.0
    return m


def inverse_peaks(kind, n, w):
    """Largest node norms of the inverse column and row passes when the
    inverse sees w[v][u] * b[v][u] (w: mask or per-coefficient weights)."""
    T = M.transform_matrix(kind, n).astype(np.float64)
    K = 2 * M.scaled_inverse(kind, n).astype(np.float64)
    t1 = np.abs(T).sum(1)
    cols = max(peak(inv, [w[v, u] * T[v] for v in range(n)], kind) * t1[u]
               for u in range(n) if w[:, u].any())
    g = np.einsum("iv,vu,va->iua", K, w, T)
    rows = peak(inv, [np.einsum("ia,b->iab", g[:, u, :], T[u]) for u in range(n)], kind)
    return cols, rows


KIND_N = [(k, n) for k in M.KINDS for n in (8, 16, 32)] + [(k, 8) for k in M.COMPARISON_KINDS]


@pytest.mark.parametrize("kind,n", KIND_N)
def test_model_computes_the_transform_and_its_inverse(kind, n):
    t = Forms()
    assert np.array_equal(np.array(fwd(unit(n), kind, t)), M.transform_matrix(kind, n))
    assert np.array_equal(np.array(inv(unit(n), kind, t)), 2 * M.scaled_inverse(kind, n))


@pytest.mark.parametrize("kind,n", KIND_N)
def test_zonal_path_fits_int32_for_full_range_int16(kind, n):
    T = M.transform_matrix(kind, n)
    row = peak(fwd, unit(n), kind)
    col = row * np.abs(T).sum(1).max()
    assert col * XMAX <= INT32
    # every r for N = 8, 16; for N = 32 a stride through the range plus the
    # levels where the inverse's intermediates peak
    rs = range(1, n * n + 1) if n < 32 else sorted(set(range(1, 1025, 37)) |
                                                    {172, 407, 692, 768, 1024})
    worst = max(max(inverse_peaks(kind, n, mask(n, r))) for r in rs)
    assert worst * XMAX <= INT32, worst
    # the bound is tight enough to mean something: full retention needs 4 N^2
    assert worst >= 4 * n * n


def round_half_away(x):
    return math.floor(abs(x) + 0.5) * (1 if x >= 0 else -1)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [16, 32])
def test_quantised_path_fits_int32_for_full_range_int16(kind, n):
    # b~ = level * DQ = 2 rho b + e with rho = MQ DQ / 2^25 and |e| <= DQ / 2;
    # the linear part has an exact bound, e is bounded term by term, and the
    # column results are halved (exactly) before the row pass
    T = M.transform_matrix(kind, n).astype(np.float64)
    d = np.diag(T @ T.T)
    forms = []

    def collect(v):
        forms.append(np.abs(v))
        return v
    outs = np.abs(np.array(inv(unit(n), kind, collect)))
    W = np.array(forms)
    for q in (1, 16, 4096):
        g = q * np.sqrt(np.outer(d, d))
        mq = np.vectorize(lambda x: round_half_away(2 ** 24 / x))(g)
        dq = np.vectorize(lambda x: round_half_away(2 * x))(g)
        rho = mq * dq / 2 ** 25
        e = dq / 2
        col_lin, _ = inverse_peaks(kind, n, 2 * rho)
        _, row_lin = inverse_peaks(kind, n, rho)
        col = col_lin * XMAX + (W @ e).max()
        row = row_lin * XMAX + (W @ ((outs @ e) / 2 + 0.5).T).max()
        assert max(col, row) <= INT32, (q, col, row)
        # 24-bit products of the dequantiser are exact
        bmax = np.abs(T).sum(1).max() ** 2 * XMAX
        assert bmax * mq.max() / 2 ** 24 + 1 < 2 ** 23 and dq.max() < 2 ** 23


@pytest.mark.parametrize("kind", M.KINDS + M.COMPARISON_KINDS)
def test_quantised_8point_path_fits_int32_for_full_range_int16(kind):
    # N = 8 keeps the dequantised values' fractional bit through both inverse
    # passes (no halving between them): bound b~ = 2 rho b + e directly
    n = 8
    T = M.transform_matrix(kind, n).astype(np.float64)
    d = np.diag(T @ T.T)
    forms = []

    def collect(v):
        forms.append(np.abs(v))
        return v
    outs = np.abs(np.array(inv(unit(n), kind, collect)))
    W = np.array(forms)
    for q in (1, 16, 4096):
        g = q * np.sqrt(np.outer(d, d))
        mq = np.vectorize(lambda x: round_half_away(2 ** 24 / x))(g)
        dq = np.vectorize(lambda x: round_half_away(2 * x))(g)
        rho = mq * dq / 2 ** 25
        e = dq / 2
        col_lin, row_lin = inverse_peaks(kind, n, 2 * rho)
        col = col_lin * XMAX + (W @ e).max()
        row = row_lin * XMAX + (W @ (outs @ e).T).max()
        assert max(col, row) <= INT32, (q, col, row)
        bmax = np.abs(T).sum(1).max() ** 2 * XMAX
        assert bmax * mq.max() / 2 ** 24 + 1 < 2 ** 23 and dq.max() < 2 ** 23


@pytest.mark.parametrize("kind", M.KINDS)
def test_64_point_level_fits_int32_for_8bit_input_only(kind):
    # the forward passes see unshifted pixels (<= 255, the shift is folded
    # into the DC coefficient), the inverse the coefficients of x - 128
    n = 64
    T = M.transform_matrix(kind, n)
    row = peak(fwd, unit(n), kind)
    assert row * np.abs(T).sum(1).max() * 255 <= INT32
    rs = (1, 10, 36, 100, 500, 1000, 2000, 3000, 4096)
    worst = max(max(inverse_peaks(kind, n, mask(n, r))) for r in rs)
    assert worst * 128 <= INT32
    # and the whole int16 range would not fit: the library refuses it at N = 64
    assert worst * XMAX > INT32


@pytest.mark.parametrize("n", [8, 16, 32])
def test_quantiser_float64_evaluation_is_exact(n):
    """The kernels evaluate level = sign(b) floor(|b| MQ / 2^24 + 1/2) as
    trunc(copysign(|b| m + 1/2, b)) in float64 with m = MQ / 2^24.  With
    |b| MQ < 2^47 (bounded above for every transform, N and step) |b| m + 1/2
    is a multiple of 2^-24 below 2^24, so it is exact in float64 and its
    truncation is the floor.  Checked here against the integer form on the
    largest |b| and MQ, on exact ties and on random pairs, with Python's
    float64 (the product and the sum are exact, as the fused multiply-add
    is)."""
    from oracle import pipeline as P
    rng = np.random.default_rng(n)
    for kind in (M.KINDS if n > 8 else M.KINDS + M.COMPARISON_KINDS):
        T = M.transform_matrix(kind, n).astype(np.float64)
        d = np.diag(T @ T.T)
        bmax = int(np.abs(T).sum(1).max() ** 2 * XMAX)
        for q in (1, 3, 16, 255, 4096):
            g = q * np.sqrt(np.outer(d, d))
            mqs = np.unique(np.vectorize(lambda x: round_half_away(2 ** 24 / x))(g)).astype(np.int64)
            assert bmax * int(mqs.max()) < 2 ** 47
            bs = np.concatenate([[0, 1, -1, bmax, -bmax], rng.integers(-bmax, bmax + 1, 2000)])
            for mq in mqs:
                m = float(mq) * 2.0 ** -24
                got = [int(math.copysign(abs(float(b)) * m + 0.5, float(b))) for b in bs]
                want = P.quantise(bs, np.full(bs.shape, mq))
                assert np.array_equal(np.array(got, dtype=np.int64), want), (kind, q, mq)
    # exact ties: |b| MQ = k 2^24 + 2^23 rounds away from zero
    for mq in (1 << 23, 3 << 22, (1 << 24) - 1):
        m = float(mq) * 2.0 ** -24
        for b in range(-4097, 4098, 7):
            want = int(P.quantise(np.array([b]), np.array([mq]))[0])
            assert int(math.copysign(abs(float(b)) * m + 0.5, float(b))) == want, (b, mq)
