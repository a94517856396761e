"""GPU parity: the HIP kernels against the CPU oracle, element by element.

Integer outputs (retained coefficients, quantiser levels, reconstructions,
error energies) must be bit-exact; the float32 scaled coefficients must be
within 1e-5 relative of the float64 oracle (exact zeros exactly zero)."""
import numpy as np
import pytest

from oracle import matrices as M
from oracle import pipeline as P
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU-only runs deselect these
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2207_11638_amd as adct  # noqa: E402

DEV = torch.device("cuda:0")
RTOL = 1e-5


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check_scaled(got, want):
    got = got.astype(np.float64)
    zero = want == 0
    assert np.all(got[zero] == 0)
    rel = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
    assert rel.size == 0 or rel.max() <= RTOL, rel.max()


def oracle_batch(imgs, kind, n, r, q):
    outs = [P.compress(im, kind, n, r, q) for im in imgs]
    return {k: np.stack([o[k] for o in outs]) for k in ("kept", "scaled", "recon")}, \
        [o["sse"] for o in outs]


def compare_compress(imgs, kind, n, r, q=0, x=None):
    if x is None:
        x = to_dev(np.stack(imgs))
    out = adct.compress(x, kind, n, r, q)
    want, sse = oracle_batch(imgs, kind, n, r, q)
    assert np.array_equal(host(out["kept"]), want["kept"])
    check_scaled(host(out["scaled"]), want["scaled"])
    rec = host(out["recon"])
    assert np.array_equal(rec.reshape(want["recon"].shape), want["recon"])
    assert host(out["sse"]).astype(np.int64).tolist() == sse
    return out


def u8_images(b, h, w, seed):
    return [synth.ar1_image(h, w, rho=0.95, seed=seed + i) for i in range(b)]


def i16_images(b, h, w, seed):
    return [synth.laplace_residual(h, w, seed=seed + i) for i in range(b)]


# ------------------------------------------------------------------ fused path
# sizes span several workgroups and end in a partial one (ragged tail)
SHAPES = {8: (40, 8 * 300), 16: (48, 16 * 37), 32: (64, 32 * 19)}


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("r", [1, 3, 6, 10, 11, 16, 28, 45, 50, 64])
def test_compress8_u8(kind, r):
    h, w = SHAPES[8]
    compare_compress(u8_images(2, h, w, 100), kind, 8, r)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("r", [1, 10, 64])
def test_compress8_i16(kind, r):
    h, w = SHAPES[8]
    compare_compress(i16_images(2, h, w, 200), kind, 8, r)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("r", [1, 6, 28, 100, "all"])
def test_compress_jam_u8(kind, n, r):
    r = n * n if r == "all" else r
    h, w = SHAPES[n]
    compare_compress(u8_images(2, h, w, 300), kind, n, r)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("dtype", ["u8", "i16"])
def test_compress_jam_kept_only(kind, n, dtype):
    """Kept coefficients without the scaled output, through every kept bound
    (4 columns for r <= 10, 8 for r <= 36, N above)."""
    h, w = SHAPES[n]
    imgs = u8_images(2, h, w, 350) if dtype == "u8" else i16_images(2, h, w, 360)
    x = to_dev(np.stack(imgs))
    for r in (1, 2, 3, 5, 6, 9, 10, 11, 15, 21, 28, 35, 36, 37, 100):
        out = adct.compress(x, kind, n, r, scaled=False)
        assert out["scaled"] is None
        want, sse = oracle_batch(imgs, kind, n, r, 0)
        assert np.array_equal(host(out["kept"]), want["kept"]), r
        rec = host(out["recon"])
        assert np.array_equal(rec.reshape(want["recon"].shape), want["recon"]), r
        assert host(out["sse"]).astype(np.int64).tolist() == sse, r


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("r", [6, "all"])
def test_compress_jam_i16(kind, n, r):
    r = n * n if r == "all" else r
    h, w = SHAPES[n]
    compare_compress(i16_images(2, h, w, 400), kind, n, r)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("q", [1, 8, 16, 33, 64, 4096])
def test_quantised_i16(kind, n, q):
    h, w = SHAPES[n]
    compare_compress(i16_images(1, h, w, 500 + q), kind, n, n * n, q)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
def test_quantised_u8_partial_retention(kind, n):
    h, w = SHAPES[n]
    compare_compress(u8_images(1, h, w, 600), kind, n, 20, 8)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
def test_extreme_images(kind, n):
    h, w = 2 * n, 5 * n
    yy, xx = np.indices((h, w))
    imgs = [np.zeros((h, w), np.uint8), np.full((h, w), 255, np.uint8),
            ((yy + xx) % 2 * 255).astype(np.uint8), ((xx // 3 + yy // 5) % 2 * 255).astype(np.uint8)]
    for r in (1, 5, n * n):
        compare_compress(imgs, kind, n, r)
    res = [np.full((h, w), 255, np.int16), np.full((h, w), -255, np.int16),
           (((yy + xx) % 2) * 510 - 255).astype(np.int16)]
    for r in (1, n * n):
        compare_compress(res, kind, n, r)
    compare_compress(res, kind, n, n * n, 1)
    compare_compress(res, kind, n, n * n, 4096)


def worst_case_tiles(kind, n, r, count=8):
    """Full-range int16 tiles that maximise |X[i][j]| of the exact inverse
    X = U mask_r(T A T^T) U^T (eqs. 6/7 and section 6.1 with U = N T^-1, the
    zig-zag mask of section 5.1): X[i][j] is the linear form
    sum_ab C_ij[a][b] A[a][b], largest at A = 32767 sign(C_ij) (-32768 where
    the sign is negative).  One tile for each of the `count` largest forms."""
    T = M.transform_matrix(kind, n).astype(np.float64)
    U = M.scaled_inverse(kind, n).astype(np.float64)
    m = np.zeros((n, n))
    for p in M.zigzag(n)[:r]:
        m[p] = 1.0
    G = np.einsum("iv,vu,va->iua", U, m, T)          # (i, u, a)
    H = np.einsum("ju,ub->jub", U, T)                # (j, u, b)
    C = (G.transpose(0, 2, 1).reshape(n * n, n) @ H.transpose(1, 0, 2).reshape(n, n * n))
    C = C.reshape(n, n, n, n).transpose(0, 2, 1, 3)  # (i, j, a, b)
    l1 = np.abs(C).sum(axis=(2, 3)).reshape(-1)
    tiles = []
    for k in np.argsort(l1)[::-1][:count]:
        s = np.sign(C[k // n, k % n])
        tiles.append(np.where(s > 0, 32767, np.where(s < 0, -32768, 0)).astype(np.int16))
    return tiles


# retention levels over the whole range, including the ones where the largest
# intermediate of the 16- and 32-point inverses peaks
WORST_R = {8: (4, 11, 31, 47, 64), 16: (37, 56, 146, 173, 256),
           32: (172, 407, 692, 768, 1024)}


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
def test_full_range_int16_worst_case(kind, n):
    # int16 inputs are exact over their whole range: every intermediate of
    # the fused path stays within int32 for any r and any step up to 4096
    for r in WORST_R[n]:
        tiles = worst_case_tiles(kind, n, r)
        row = np.concatenate(tiles, axis=1)
        img = np.concatenate([row, (-row.astype(np.int32)).clip(-32768, 32767).astype(np.int16)])
        compare_compress([img], kind, n, r)
        if r == n * n:
            for q in (1, 16, 4096):
                compare_compress([img], kind, n, r, q)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_strided_geometry(n):
    # pitch > width and image stride > pitch * height, through tensor views
    b, h, w = 3, 2 * n, 7 * n
    full = np.zeros((b, h + 3, w + 48), np.uint8)
    imgs = u8_images(b, h, w, 700)
    for i in range(b):
        full[i, :h, :w] = imgs[i]
    xd = to_dev(full)[:, :h, :w]
    compare_compress(imgs, M.ROUND, n, 10, x=xd)


def test_outputs_are_optional():
    imgs = u8_images(1, 16, 64, 800)
    x = to_dev(np.stack(imgs))
    want, sse = oracle_batch(imgs, M.SIGN, 8, 10, 0)
    out = adct.compress(x, M.SIGN, 8, 10, kept=False, scaled=False, recon=False)
    assert host(out["sse"]).tolist() == sse
    out = adct.compress(x, M.SIGN, 8, 10, recon=False, sse=False)
    assert np.array_equal(host(out["kept"]), want["kept"])


def test_sse_accumulates():
    imgs = u8_images(2, 16, 64, 900)
    x = to_dev(np.stack(imgs))
    sse = torch.zeros(2, dtype=torch.uint64, device=DEV)
    adct.compress(x, M.ROUND, 8, 6, kept=False, scaled=False, recon=False, sse=sse)
    adct.compress(x, M.ROUND, 8, 6, kept=False, scaled=False, recon=False, sse=sse)
    _, want = oracle_batch(imgs, M.ROUND, 8, 6, 0)
    assert host(sse).tolist() == [2 * v for v in want]


# ------------------------------------------------------- forward / inverse only
@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("dt", ["u8", "i16"])
def test_fwd2d(kind, n, dt):
    h, w = SHAPES[n]
    imgs = u8_images(2, h, w, 1000) if dt == "u8" else i16_images(2, h, w, 1000)
    got = host(adct.fwd2d(to_dev(np.stack(imgs)), kind, n))
    want = np.stack([P.forward2d(im, kind, n) for im in imgs])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("r", [1, 10, "all"])
def test_inv2d_roundtrip(kind, n, r):
    r = n * n if r == "all" else r
    h, w = SHAPES[n]
    imgs = u8_images(2, h, w, 1100)
    coef = adct.fwd2d(to_dev(np.stack(imgs)), kind, n)
    rec = host(adct.inv2d(coef, kind, n, r))
    want = np.stack([P.compress(im, kind, n, r)["recon"] for im in imgs])
    assert np.array_equal(rec, want)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
def test_inv2d_quantised_levels(kind, n):
    h, w = SHAPES[n]
    res = i16_images(1, h, w, 1200)[0]
    q = 16
    mq, dq = P.quant_tables(kind, n, q)
    levels = P.quantise(P.forward2d(res, kind, n), mq)
    coef = to_dev(levels.astype(np.int32)[None])
    rec = host(adct.inv2d(coef, kind, n, n * n, q, dtype=torch.int16))
    want = P.inverse2d(P.dequantise(levels, dq), kind, n, np.int16, P.QUANT_FRAC)
    assert np.array_equal(rec[0], want)


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("rq", [(1, 0), (13, 0), ("all", 0), ("all", 24)])
def test_decompress_equals_compress_recon(kind, n, rq):
    r, q = rq
    r = n * n if r == "all" else r
    h, w = SHAPES[n]
    imgs = i16_images(2, h, w, 1300) if q else u8_images(2, h, w, 1300)
    x = to_dev(np.stack(imgs))
    out = adct.compress(x, kind, n, r, q)
    rec = adct.decompress(out["kept"], kind, n, r, q, dtype=x.dtype)
    assert np.array_equal(host(rec), host(out["recon"]))


def test_empty_batch_is_a_no_op():
    x = torch.zeros((0, 16, 16), dtype=torch.uint8, device=DEV)
    out = adct.compress(x, M.SIGN, 8, 10)
    torch.cuda.synchronize()
    assert out["kept"].numel() == 0


def test_repeatable():
    imgs = u8_images(1, 64, 256, 1400)
    x = to_dev(np.stack(imgs))
    a = adct.compress(x, M.ROUND, 16, 28)
    b = adct.compress(x, M.ROUND, 16, 28)
    for k in ("kept", "scaled", "recon", "sse"):
        assert np.array_equal(host(a[k]), host(b[k]))


# ------------------------------------------------- int8 matrix-core engine (N=8)
def compare_compress_mfma(imgs, kind, r, x=None):
    if x is None:
        x = to_dev(np.stack(imgs))
    out = adct.compress(x, kind, 8, r, engine="mfma")
    want, sse = oracle_batch(imgs, kind, 8, r, 0)
    assert np.array_equal(host(out["kept"]), want["kept"])
    check_scaled(host(out["scaled"]), want["scaled"])
    rec = host(out["recon"])
    assert np.array_equal(rec.reshape(want["recon"].shape), want["recon"])
    assert host(out["sse"]).astype(np.int64).tolist() == sse
    return out


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("r", [1, 3, 6, 10, 11, 16, 28, 45, 50, 64])
def test_mfma_matches_oracle(kind, r):
    # 300 tiles per row: four full waves of 64 tiles and a partial one, whose
    # last 16-tile step is partial as well
    h, w = SHAPES[8]
    compare_compress_mfma(u8_images(2, h, w, 300), kind, r)


@pytest.mark.parametrize("kind", M.KINDS)
def test_mfma_equals_butterflies_on_extremes(kind):
    # saturated content drives the coefficients and the reconstruction to
    # their limits (|b| up to 8192, clipping at 0 and 255)
    rng = synth.rng_for(77)
    imgs = [rng.choice(np.array([0, 255], dtype=np.uint8), size=(32, 8 * 70)) for _ in range(2)]
    imgs.append(np.full((32, 8 * 70), 255, dtype=np.uint8))
    imgs.append(np.zeros((32, 8 * 70), dtype=np.uint8))
    x = to_dev(np.stack(imgs))
    for r in (1, 10, 37, 64):
        a = adct.compress(x, kind, 8, r, engine="mfma")
        b = adct.compress(x, kind, 8, r)
        for key in ("kept", "scaled", "recon", "sse"):
            assert torch.equal(a[key], b[key]), (key, r)
    compare_compress_mfma(imgs, kind, 45, x=x)


def test_mfma_pitched_batch_and_partial_outputs():
    imgs = u8_images(3, 24, 8 * 21, 400)
    full = np.zeros((3, 24, 8 * 21 + 40), dtype=np.uint8)
    full[:, :, : 8 * 21] = np.stack(imgs)
    x = to_dev(full)[:, :, : 8 * 21]
    compare_compress_mfma(imgs, 2, 21, x=x)
    # only the reconstruction, only the coefficients
    a = adct.compress(x, 1, 8, 10, engine="mfma", kept=False, scaled=False, sse=False)
    b = adct.compress(x, 1, 8, 10, kept=False, scaled=False, sse=False)
    assert torch.equal(a["recon"], b["recon"])
    a = adct.compress(x, 1, 8, 10, engine="mfma", recon=False, sse=False)
    b = adct.compress(x, 1, 8, 10, recon=False, sse=False)
    assert torch.equal(a["kept"], b["kept"]) and torch.equal(a["scaled"], b["scaled"])


def test_mfma_rejects_what_it_does_not_cover():
    x = to_dev(np.stack(u8_images(1, 16, 16, 1)))
    with pytest.raises(ValueError):
        adct.compress(x, 1, 16, 10, engine="mfma")
    with pytest.raises(ValueError):
        adct.compress(x, 1, 8, 10, 16, engine="mfma")
