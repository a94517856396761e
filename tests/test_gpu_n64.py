"""GPU parity of the 64-point level of the Chen-JAM recursion (section 6.1):
8-bit images, zonal retention, bit-exact against the oracle; moments and
coding gains at N = 64; the cases the library refuses at this size."""
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

from test_gpu_parity import compare_compress, host, to_dev  # noqa: E402

# three tile rows, 13 tiles per row: several workgroups of 4 tiles, a partial one
H, W = 64 * 3, 64 * 13


def images(b, seed):
    return [synth.ar1_image(H, W, rho=0.95, seed=seed + i) for i in range(b)]


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("r", [1, 10, 11, 36, 37, 100, 1000, 4096])
def test_compress64(kind, r):
    compare_compress(images(2, 5000), kind, 64, r)


@pytest.mark.parametrize("kind", M.KINDS)
def test_extreme_images_64(kind):
    yy, xx = np.indices((64, 128))
    imgs = [np.zeros((64, 128), np.uint8), np.full((64, 128), 255, np.uint8),
            ((yy + xx) % 2 * 255).astype(np.uint8)]
    for r in (1, 50, 4096):
        compare_compress(imgs, kind, 64, r)


@pytest.mark.parametrize("kind", M.KINDS)
def test_fwd_inv_decompress_64(kind):
    imgs = images(1, 5100)
    x = to_dev(np.stack(imgs))
    coef = adct.fwd2d(x, kind, 64)
    assert np.array_equal(host(coef)[0], P.forward2d(imgs[0], kind, 64))
    for r in (6, 4096):
        want = P.compress(imgs[0], kind, 64, r)["recon"]
        assert np.array_equal(host(adct.inv2d(coef, kind, 64, r))[0], want)
        out = adct.compress(x, kind, 64, r)
        assert np.array_equal(host(adct.decompress(out["kept"], kind, 64, r))[0], want)


@pytest.mark.parametrize("kind", M.KINDS)
def test_quality_measures_64(kind):
    img = images(1, 5200)[0]
    mom = host(adct.moments(to_dev(img), kind, 64))[0]
    want = P.coefficient_moments(img, kind, 64)
    nn = 64 * 64
    rec = [int(v) for v in mom]
    s1 = [(v - (1 << 64)) if v >= (1 << 63) else v for v in rec[:nn]]
    assert s1 == [int(v) for v in want["s1"].reshape(-1)]
    assert [rec[2 * nn + p] * (1 << 32) + rec[nn + p] for p in range(nn)] == \
        [int(v) for v in want["s2"].reshape(-1)]
    got = host(adct.coding_gain(adct.moments(to_dev(img), kind, 64), kind, 64, "cols"))[0]
    want_cg = P.empirical_coding_gain(img, kind, 64, "cols")
    assert abs(got - want_cg) <= 1e-5 * max(abs(want_cg), 1.0)
    rho = np.array([0.0, 0.5, 0.9, 0.95, 0.99], dtype=np.float32)
    cg, klt = adct.coding_gain_ar1(to_dev(rho), kind, 64, "cols")
    cg, klt = host(cg), host(klt)
    c = M.near_orthogonal(kind, 64)
    for i, p in enumerate(rho.astype(np.float64)):
        w = MT.coding_gain(c, p, "cols")
        assert abs(cg[i] - w) <= 1e-5 * max(abs(w), 1.0), (p, cg[i], w)
        wk = MT.klt_coding_gain(64, p)
        assert abs(klt[i] - wk) <= 1e-5 * max(abs(wk), 1.0)


def test_64_point_refuses_int16_and_quantisation():
    x8 = to_dev(np.zeros((64, 64), np.uint8))
    x16 = to_dev(np.zeros((64, 64), np.int16))
    with pytest.raises(adct.AdctError):
        adct.compress(x16, 1, 64, 10)
    with pytest.raises(adct.AdctError):
        adct.compress(x8, 2, 64, 4096, 16)
    with pytest.raises(adct.AdctError):
        adct.compress(x8, adct.ADCT_WHT, 64, 10)
