"""GPU parity of the 8-point comparison transforms of section 4 (WHT, SDCT,
HT) through the same fused kernels as the proposed transforms: bit-exact
integer outputs, float32 scaled coefficients within 1e-5 relative of the
oracle, on sizes that span several waves and end in a partial one."""
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

from test_gpu_parity import (DEV, check_scaled, compare_compress, compare_compress_mfma,  # noqa: E402
                             host, to_dev, worst_case_tiles)

H, W = 40, 8 * 300
KINDS = M.COMPARISON_KINDS


def u8_images(b, seed):
    return [synth.ar1_image(H, W, rho=0.95, seed=seed + i) for i in range(b)]


def i16_images(b, seed):
    return [synth.laplace_residual(H, W, seed=seed + i) for i in range(b)]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("r", [1, 6, 10, 16, 28, 45, 64])
def test_compress_u8(kind, r):
    compare_compress(u8_images(2, 3100), kind, 8, r)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rq", [(1, 0), (64, 0), (64, 1), (64, 16), (64, 4096), (20, 8)])
def test_compress_i16(kind, rq):
    r, q = rq
    compare_compress(i16_images(1, 3200 + r + q), kind, 8, r, q)


@pytest.mark.parametrize("kind", KINDS)
def test_full_range_int16_worst_case(kind):
    for r in (4, 11, 31, 47, 64):
        row = np.concatenate(worst_case_tiles(kind, 8, r), axis=1)
        img = np.concatenate([row, (-row.astype(np.int32)).clip(-32768, 32767).astype(np.int16)])
        compare_compress([img], kind, 8, r)
        if r == 64:
            for q in (1, 16, 4096):
                compare_compress([img], kind, 8, r, q)


@pytest.mark.parametrize("kind", KINDS)
def test_extreme_u8_images(kind):
    yy, xx = np.indices((16, 40))
    imgs = [np.zeros((16, 40), np.uint8), np.full((16, 40), 255, np.uint8),
            ((yy + xx) % 2 * 255).astype(np.uint8)]
    for r in (1, 5, 64):
        compare_compress(imgs, kind, 8, r)


@pytest.mark.parametrize("kind", KINDS)
def test_fwd2d_inv2d_decompress(kind):
    imgs = u8_images(2, 3300)
    x = to_dev(np.stack(imgs))
    coef = adct.fwd2d(x, kind, 8)
    assert np.array_equal(host(coef), np.stack([P.forward2d(im, kind, 8) for im in imgs]))
    for r in (1, 10, 64):
        want = np.stack([P.compress(im, kind, 8, r)["recon"] for im in imgs])
        assert np.array_equal(host(adct.inv2d(coef, kind, 8, r)), want)
        out = adct.compress(x, kind, 8, r)
        assert np.array_equal(host(adct.decompress(out["kept"], kind, 8, r)), want)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("r", [1, 10, 45, 64])
def test_mfma_engine(kind, r):
    compare_compress_mfma(u8_images(1, 3400), kind, r)


@pytest.mark.parametrize("kind", KINDS)
def test_quality_measures(kind):
    imgs = u8_images(2, 3500)
    mom = adct.moments(to_dev(np.stack(imgs)), kind, 8)
    cg = host(adct.coding_gain(mom, kind, 8, "cols"))
    for i, im in enumerate(imgs):
        want = P.empirical_coding_gain(im, kind, 8, "cols")
        assert abs(cg[i] - want) <= 1e-5 * max(abs(want), 1.0), (cg[i], want)
    rho = np.array([0.0, 0.5, 0.9, 0.95, 0.99], dtype=np.float32)
    got, _ = adct.coding_gain_ar1(to_dev(rho), kind, 8, "cols")
    got = host(got)
    from oracle import metrics as MT
    c = M.near_orthogonal(kind, 8)
    for i, p in enumerate(rho.astype(np.float64)):
        want = MT.coding_gain(c, p, "cols")
        assert abs(got[i] - want) <= 1e-5 * max(abs(want), 1.0), (p, got[i], want)


def test_comparison_transforms_are_8_point_only():
    x = to_dev(np.zeros((16, 16), np.uint8))
    for kind in KINDS:
        with pytest.raises(adct.AdctError):
            adct.compress(x, kind, 16, 10)


def test_ordering_of_reconstruction_quality():
    """Section 4 orders the transforms by closeness to the DCT: on smooth
    AR(1) images at r = 10 the round-based T^8 keeps more energy than the
    sign-based T~8, which beats SDCT and WHT (error energies 1.79, 3.64, 3.32,
    5.05; HT, 47.61, is far behind).  Checked on the library's PSNR."""
    img = synth.ar1_image(512, 512, rho=0.95, seed=0)
    x = to_dev(img)
    psnr = {}
    for kind in M.KINDS + KINDS:
        out = adct.compress(x, kind, 8, 10)
        psnr[kind] = float(host(adct.psnr(out["sse"], img.size))[0])
        want = P.compress(img, kind, 8, 10)["psnr"]
        assert abs(psnr[kind] - want) <= 1e-5 * abs(want)
    assert psnr[M.ROUND] > psnr[M.SIGN] and psnr[M.ROUND] > psnr[M.SDCT]
    assert psnr[M.WHT] > psnr[M.HT] and psnr[M.SDCT] > psnr[M.HT]


# ------------------------------------------------- the exact DCT in float32
def check_dct(imgs, r, out):
    """Float32 DCT against the float64 oracle.  Coefficients: per tile,
    max |c - c64| <= 1e-5 * ||A||_2 (the tile's energy, equal to that of its
    coefficients); reconstruction: exact except where the float64 value lies
    within 1e-2 of a rounding tie, where either neighbour is accepted; error
    energy: exactly the one of the kernel's own reconstruction, and within the
    ambiguous pixels' slack of the oracle's; PSNR within 1e-5 relative."""
    sc = host(out["scaled"]).astype(np.float64)
    rec = host(out["recon"])
    sse = host(out["sse"]).astype(np.int64)
    for i, im in enumerate(imgs):
        want = P.compress_dct(im, r)
        a = P.to_tiles(P.level_shift(im), 8).astype(np.float64)
        norm = np.sqrt((a ** 2).sum(axis=(2, 3)))[..., None]
        err = np.abs(sc[i] - want["scaled"])
        assert np.all(err <= 1e-5 * np.maximum(norm, 1.0)), err.max()
        amb = want["margin"] < 1e-2
        diff = rec[i].astype(np.int64) - want["recon"].astype(np.int64)
        assert np.all(diff[~amb] == 0)
        assert np.all(np.abs(diff[amb]) <= 1)
        own = int(((rec[i].astype(np.int64) - im.astype(np.int64)) ** 2).sum())
        assert sse[i] == own
        slack = int((2 * np.abs(im.astype(np.int64) - want["recon"].astype(np.int64))[amb] + 1).sum())
        assert abs(own - want["sse"]) <= slack
        if want["sse"]:
            got_p = 10 * np.log10(255.0 ** 2 * im.size / own) if own else np.inf
            assert abs(got_p - want["psnr"]) <= 1e-5 * abs(want["psnr"]) or amb.any()


@pytest.mark.parametrize("r", [1, 6, 10, 15, 28, 45, 64])
def test_dct_float32_u8(r):
    imgs = u8_images(2, 3600)
    out = adct.compress(to_dev(np.stack(imgs)), adct.ADCT_DCT, 8, r)
    assert out["kept"] is None
    check_dct(imgs, r, out)


@pytest.mark.parametrize("r", [1, 10, 64])
def test_dct_float32_i16(r):
    imgs = i16_images(1, 3700)
    out = adct.compress(to_dev(np.stack(imgs)), adct.ADCT_DCT, 8, r)
    check_dct(imgs, r, out)


def test_dct_psnr_and_ape():
    """The reference PSNR of section 5 and the absolute percentage error of
    the approximations relative to it (section 5.1), on one 512 x 512 image."""
    img = synth.ar1_image(512, 512, rho=0.95, seed=0)
    x = to_dev(img)
    ref = adct.compress_quality(x, adct.ADCT_DCT, 8, 10)
    assert ref["kept"] is None and ref["coding_gain"] is None
    want = P.compress_dct(img, 10)["psnr"]
    got = float(host(ref["psnr"])[0])
    assert abs(got - want) <= 1e-5 * want
    for kind in M.KINDS:
        p = float(host(adct.compress_quality(x, kind, 8, 10)["psnr"])[0])
        ape = 100.0 * abs(p - got) / got
        want_ape = 100.0 * abs(P.compress(img, kind, 8, 10)["psnr"] - want) / want
        assert abs(ape - want_ape) <= 1e-3


def test_dct_rejects_integer_only_requests():
    x = to_dev(np.zeros((8, 8), np.uint8))
    kept = torch.empty((1, 1, 1, 10), dtype=torch.int32, device=DEV)
    with pytest.raises(adct.AdctError):
        adct.compress(x, adct.ADCT_DCT, 8, 10, kept=kept)
    with pytest.raises(adct.AdctError):
        adct.compress(x, adct.ADCT_DCT, 8, 10, 16)
    with pytest.raises(adct.AdctError):
        adct.fwd2d(x, adct.ADCT_DCT, 8)
    with pytest.raises(adct.AdctError):
        adct.compress(to_dev(np.zeros((16, 16), np.uint8)), adct.ADCT_DCT, 16, 10)
