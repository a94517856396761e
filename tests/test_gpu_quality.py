"""GPU parity of the quality measures: coefficient moments (bit-exact), the
measured 2D coding gain, the AR(1) coding gain and PSNR (float32 within
1e-5 relative of the float64 oracle).

Tolerance of the float32 gains: |got - want| <= 1e-5 * max(|want|, 1 dB).  A
coding gain can cross zero (a non-orthogonal transform at rho -> 0), where
no relative bound is attainable; above 1 dB in magnitude the bound is the
plain 1e-5 relative one."""
import numpy as np
import pytest

from oracle import matrices as M
from oracle import metrics as MT
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


def close(got, want):
    return abs(float(got) - float(want)) <= RTOL * max(abs(float(want)), 1.0)


def record_matches(rec, mom, n):
    """A device moment record against the oracle's exact sums."""
    nn = n * n
    rec = [int(v) for v in rec]
    s1 = [(v - (1 << 64)) if v >= (1 << 63) else v for v in rec[:nn]]
    s2 = [rec[2 * nn + p] * (1 << 32) + rec[nn + p] for p in range(nn)]
    a1 = rec[3 * nn + 2]
    a1 = a1 - (1 << 64) if a1 >= (1 << 63) else a1
    return (s1 == [int(v) for v in mom["s1"].reshape(-1)] and
            s2 == [int(v) for v in mom["s2"].reshape(-1)] and
            rec[3 * nn] == mom["tiles"] and rec[3 * nn + 1] == mom["pixels"] and
            a1 == mom["a1"] and rec[3 * nn + 3] == mom["a2"])


# shapes: several workgroups per tile row with a partial last group, and
# more tile groups than the walking workgroups of one image
SHAPES = {8: (72, 8 * 75), 16: (80, 16 * 21), 32: (96, 32 * 11)}


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("dtype", ["u8", "i16"])
def test_moments_match_oracle(kind, n, dtype):
    h, w = SHAPES[n]
    if dtype == "u8":
        imgs = [synth.ar1_image(h, w, rho=0.9 + 0.03 * i, seed=500 + i) for i in range(3)]
    else:
        imgs = [synth.laplace_residual(h, w, seed=600 + i) for i in range(3)]
    mom = host(adct.moments(to_dev(np.stack(imgs)), kind, n))
    for i, im in enumerate(imgs):
        assert record_matches(mom[i], P.coefficient_moments(im, kind, n), n), (i, kind, n)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_moments_full_int16_range(n):
    """Tiles of +-32767 / -32768: the squares use their high halves."""
    rng = np.random.default_rng(7)
    h, w = 2 * n, 5 * n
    img = np.where(rng.random((h, w)) < 0.5, -32768, 32767).astype(np.int16)
    img[:n, :n] = 32767
    for kind in M.KINDS:
        mom = host(adct.moments(to_dev(img), kind, n))
        assert record_matches(mom[0], P.coefficient_moments(img, kind, n), n)


@pytest.mark.parametrize("kind", M.KINDS + M.COMPARISON_KINDS)
def test_moments_extreme_u8_full_groups(kind):
    """All-0 and all-255 images whose tile rows hold full 64-tile groups: at
    the DC position 64 tiles of |b| = 128 * 64 square to 2^32 in sum, which
    a 32-bit accumulator would wrap."""
    w = 8 * 64 * 3 + 24
    imgs = [np.zeros((16, w), np.uint8), np.full((16, w), 255, np.uint8)]
    yy, xx = np.indices((16, w))
    imgs.append(((yy + xx) % 2 * 255).astype(np.uint8))
    mom = host(adct.moments(to_dev(np.stack(imgs)), kind, 8))
    for i, im in enumerate(imgs):
        assert record_matches(mom[i], P.coefficient_moments(im, kind, 8), 8), (i, kind)


@pytest.mark.parametrize("kind", M.KINDS + M.COMPARISON_KINDS)
def test_moments_8bit_narrow_images_and_many_images(kind):
    """8-bit moments of 8x8 tiles (the matrix-core form): images narrower
    than one 16-tile step (1, 3 and 17 tiles wide), a single tile row, and a
    batch of 300 images, where the walking waves per image clamp to the
    image's one tile group."""
    for h, w in ((8, 8), (8, 24), (24, 8), (8, 136), (40, 8 * 17)):
        imgs = [synth.ar1_image(h, w, rho=0.9, seed=900 + i) for i in range(2)]
        mom = host(adct.moments(to_dev(np.stack(imgs)), kind, 8))
        for i, im in enumerate(imgs):
            assert record_matches(mom[i], P.coefficient_moments(im, kind, 8), 8), (h, w, i)
    imgs = [synth.ar1_image(8, 64, rho=0.5 + 0.001 * i, seed=950 + i) for i in range(300)]
    mom = host(adct.moments(to_dev(np.stack(imgs)), kind, 8))
    for i in (0, 1, 150, 299):
        assert record_matches(mom[i], P.coefficient_moments(imgs[i], kind, 8), 8), i


def test_moments_accumulate_over_calls():
    img = synth.ar1_image(64, 256, rho=0.95, seed=11)
    x = to_dev(img)
    out = adct.moments(x, 2, 8)
    adct.moments(x, 2, 8, out=out)
    got = host(out)[0].astype(object)
    once = host(adct.moments(x, 2, 8))[0].astype(object)
    assert all(int(a) == (2 * int(b)) % (1 << 64) for a, b in zip(got, once))


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("basis", ["rows", "cols"])
def test_measured_coding_gain(kind, n, basis):
    h, w = SHAPES[n]
    imgs = [synth.ar1_image(h, w, rho=rho, seed=700 + i) for i, rho in enumerate((0.85, 0.95, 0.98))]
    imgs.append(synth.laplace_residual(h, w, seed=710).astype(np.int16))
    for im in imgs:
        mom = adct.moments(to_dev(im), kind, n)
        got = host(adct.coding_gain(mom, kind, n, basis))[0]
        want = P.empirical_coding_gain(im, kind, n, basis)
        assert close(got, want), (got, want, im.dtype)


def test_measured_coding_gain_edge_cases():
    # every tile identical: each coefficient is constant -> +inf
    tile = synth.ar1_image(8, 8, rho=0.9, seed=3)
    img = np.tile(tile, (6, 9))
    got = host(adct.coding_gain(adct.moments(to_dev(img), 1, 8), 1, 8))[0]
    assert np.isinf(got) and got > 0
    assert np.isinf(P.empirical_coding_gain(img, 1, 8))
    # constant image: the pixel variance is zero -> NaN
    flat = np.full((16, 32), 77, dtype=np.uint8)
    got = host(adct.coding_gain(adct.moments(to_dev(flat), 2, 8), 2, 8))[0]
    assert np.isnan(got) and np.isnan(P.empirical_coding_gain(flat, 2, 8))
    # an empty record (all zero) -> NaN
    empty = torch.zeros((1, 3 * 64 + 4), dtype=torch.uint64, device=DEV)
    assert np.isnan(host(adct.coding_gain(empty, 1, 8))[0])


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("basis", ["rows", "cols"])
def test_ar1_coding_gain(kind, n, basis):
    rhos = np.array([0.0, 0.05, 0.3, 0.5, 0.75, 0.85, 0.9, 0.95, 0.98, 0.99, 0.995, 0.999],
                    dtype=np.float32)
    cg, klt = adct.coding_gain_ar1(to_dev(rhos), kind, n, basis)
    cg, klt = host(cg), host(klt)
    c = M.near_orthogonal(kind, n)
    for i, rho in enumerate(rhos.astype(np.float64)):
        want = MT.coding_gain(c, rho, basis)
        assert close(cg[i], want), (rho, cg[i], want)
        want_klt = MT.klt_coding_gain(n, rho)
        assert close(klt[i], want_klt), (rho, klt[i], want_klt)


def test_ar1_coding_gain_sweep_many_values():
    """A long sweep (many workgroups) over rho in [0, 1)."""
    rhos = np.linspace(0.0, 0.999, 2001, dtype=np.float32)
    cg, klt = adct.coding_gain_ar1(to_dev(rhos), 2, 8, "cols")
    cg, klt = host(cg), host(klt)
    c = M.near_orthogonal(2, 8)
    for i in range(0, len(rhos), 97):
        rho = float(rhos[i])
        assert close(cg[i], MT.coding_gain(c, rho, "cols"))
        assert close(klt[i], MT.klt_coding_gain(8, rho))


@pytest.mark.parametrize("n", [8, 16, 32])
def test_psnr_matches_oracle(n):
    h, w = SHAPES[n]
    imgs = [synth.ar1_image(h, w, rho=0.95, seed=800 + i) for i in range(4)]
    x = to_dev(np.stack(imgs))
    out = adct.compress(x, 2, n, 10)
    ps = host(adct.psnr(out["sse"], h * w))
    for i, im in enumerate(imgs):
        want = P.compress(im, 2, n, 10)
        assert close(ps[i], want["psnr"]), (ps[i], want["psnr"])
    full = adct.compress(x, 1, n, n * n)
    assert np.all(np.isinf(host(adct.psnr(full["sse"], h * w))))


def test_quality_calls_reject_bad_arguments():
    rho = to_dev(np.array([0.5], dtype=np.float32))
    with pytest.raises(ValueError):
        adct.coding_gain_ar1(rho, 1, 8, "diagonal")
    with pytest.raises(adct.AdctError):
        adct.coding_gain_ar1(rho, 6, 8)
    with pytest.raises(adct.AdctError):
        adct.moments(to_dev(np.zeros((12, 16), np.uint8)), 1, 8)   # 12 rows: not a multiple of 8


@pytest.mark.parametrize("kind,n,dtype,r,q", [(1, 8, "u8", 10, 0), (2, 16, "u8", 28, 0),
                                              (2, 32, "i16", 1024, 16), (3, 8, "u8", 6, 0)])
def test_compress_quality_matches_oracle(kind, n, dtype, r, q):
    h, w = SHAPES[n]
    if dtype == "u8":
        imgs = [synth.ar1_image(h, w, rho=0.9, seed=900 + i) for i in range(3)]
    else:
        imgs = [synth.laplace_residual(h, w, seed=910 + i) for i in range(3)]
    x = to_dev(np.stack(imgs))
    out = adct.compress_quality(x, kind, n, r, q)
    kept, rec = host(out["kept"]), host(out["recon"])
    ps, cg = host(out["psnr"]), host(out["coding_gain"])
    for i, im in enumerate(imgs):
        want = P.compress(im, kind, n, r, q)
        assert np.array_equal(kept[i], want["kept"])
        assert np.array_equal(rec[i], want["recon"])
        assert close(ps[i], want["psnr"]), (ps[i], want["psnr"])
        want_cg = P.empirical_coding_gain(im, kind, n, "cols")
        assert close(cg[i], want_cg), (cg[i], want_cg)
    # the same outputs as the separate calls
    sep = adct.compress(x, kind, n, r, q)
    assert np.array_equal(host(sep["kept"]), kept)
    assert np.array_equal(host(adct.psnr(sep["sse"], h * w)), ps)


def test_compress_quality_workspace_checks():
    from paper_2207_11638_amd import _lib
    import ctypes as C
    lib = _lib.load()
    x = to_dev(synth.ar1_image(16, 64, seed=1))
    need = lib.adct_compress_quality_workspace(8, 1, 1)
    assert need == 8 * (1 + 3 * 64 + 4)
    work = torch.zeros(need // 8, dtype=torch.uint64, device=DEV)
    psnr = torch.zeros(1, dtype=torch.float32, device=DEV)
    cg = torch.zeros(1, dtype=torch.float32, device=DEV)
    args = [1, 8, 10, 0, C.c_void_p(x.data_ptr()), 0, 1, 16, 64, 64, 16 * 64, None, None, None,
            C.c_void_p(psnr.data_ptr()), C.c_void_p(cg.data_ptr()), 1,
            C.c_void_p(work.data_ptr())]
    assert lib.adct_compress_quality(*args, need - 8, None) == -5      # too small
    assert lib.adct_compress_quality(*args[:15], None, 1, C.c_void_p(work.data_ptr()), 8,
                                     None) == 0                        # PSNR only: one word
    assert lib.adct_compress_quality(*args, need, None) == 0
    torch.cuda.synchronize()
    want = P.compress(host(x), 1, 8, 10)
    assert close(host(psnr)[0], want["psnr"])


# ------------------------------------------------------------- SSIM and APE
@pytest.mark.parametrize("h,w", [(64, 80), (75, 201), (11, 11), (130, 70)])
def test_ssim_matches_oracle(h, w):
    """Mean SSIM of an image and its reconstructions (r = 1, 10 and exact)
    against the float64 oracle; windows span several workgroups with ragged
    edges in both directions."""
    img = synth.ar1_image(h, w, rho=0.93, seed=h + w)
    x = to_dev(np.stack([img, img, img]))
    recs = []
    for r in (1, 10, 64):
        recs.append(P.compress(img, 2, 8, r)["recon"] if h % 8 == 0 and w % 8 == 0 else
                    np.clip(img.astype(np.int16) + np.random.default_rng(r).integers(
                        -r // 4 - 1, r // 4 + 2, size=img.shape), 0, 255).astype(np.uint8))
    y = to_dev(np.stack(recs))
    got = host(adct.ssim(x, y))
    for i, rec in enumerate(recs):
        want = MT.mean_ssim(img, rec)
        assert close(got[i], want), (got[i], want)


def test_ssim_identical_and_constant_images():
    img = synth.ar1_image(40, 48, rho=0.9, seed=9)
    x = to_dev(img)
    assert abs(float(host(adct.ssim(x, x))[0]) - 1.0) <= 1e-6
    a = to_dev(np.full((24, 24), 200, np.uint8))
    b = to_dev(np.full((24, 24), 10, np.uint8))
    c1 = (0.01 * 255) ** 2
    want = (2 * 200 * 10 + c1) / (200 ** 2 + 10 ** 2 + c1)
    assert close(host(adct.ssim(a, b))[0], want)


def test_ssim_and_ape_of_the_still_image_experiment():
    """Section 5.1 on one 512 x 512 AR(1) image: PSNR and SSIM of T1 and T2
    reconstructions at r = 6, and their APE relative to the exact DCT."""
    img = synth.ar1_image(512, 512, rho=0.95, seed=0)
    x = to_dev(img)
    ref = adct.compress(x, adct.ADCT_DCT, 8, 6, scaled=False)
    ref_ssim = adct.ssim(x, ref["recon"])
    want_ref = MT.mean_ssim(img, P.compress_dct(img, 6)["recon"])
    assert abs(float(host(ref_ssim)[0]) - want_ref) <= 1e-4   # float32 DCT: ties may round apart
    for kind in M.KINDS:
        out = adct.compress(x, kind, 8, 6, scaled=False)
        s = adct.ssim(x, out["recon"])
        want = MT.mean_ssim(img, P.compress(img, kind, 8, 6)["recon"])
        assert close(host(s)[0], want)
        ape = host(adct.ape(s, ref_ssim))[0]
        want_ape = MT.absolute_percentage_error(want, float(host(ref_ssim)[0]))
        assert abs(ape - want_ape) <= 1e-4 * max(want_ape, 1.0)


def test_ssim_rejects_small_images():
    x = to_dev(np.zeros((10, 40), np.uint8))
    with pytest.raises(adct.AdctError):
        adct.ssim(x, x)
