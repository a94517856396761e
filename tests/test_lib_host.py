"""CPU checks of the HIP library: it loads, exports every declared entry point,
its host-side queries agree with the oracle, and argument errors are reported
before any GPU work (no compute calls here)."""
import ctypes as C

import numpy as np
import pytest

from oracle import matrices as M
from oracle import pipeline as P
import paper_2207_11638_amd as adct
from paper_2207_11638_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _lib.header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert lib.adct_version() >= 1


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_library_butterflies_compute_the_paper_matrices(kind, n):
    # the forward butterfly applied to unit vectors reproduces T_N, and the
    # inverse butterfly reproduces U_N = N T_N^-1
    assert np.array_equal(adct.get_matrix(kind, n), M.transform_matrix(kind, n))
    assert np.array_equal(adct.get_matrix(kind, n, inverse=True), M.scaled_inverse(kind, n))


@pytest.mark.parametrize("kind", M.COMPARISON_KINDS)
def test_library_butterflies_compute_the_comparison_matrices(kind, lib):
    # WHT, SDCT and HT of section 4: the add-only butterflies reproduce the
    # matrices and their exact integer inverses 8 T^-1; they are 8-point only
    assert np.array_equal(adct.get_matrix(kind, 8), M.transform_matrix(kind, 8))
    assert np.array_equal(adct.get_matrix(kind, 8, inverse=True), M.scaled_inverse(kind, 8))
    out = np.zeros(256, dtype=np.int32)
    assert lib.adct_get_matrix(kind, 16, 0, out.ctypes.data) == -1
    assert np.allclose(adct.scale_vector(kind, 8), M.scale_vector(kind, 8), rtol=0, atol=0)


@pytest.mark.parametrize("n", M.SIZES)
def test_zigzag_table(n):
    want = [v * n + u for v, u in M.zigzag(n)]
    assert adct.zigzag(n).tolist() == want


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
def test_scale_vector(kind, n):
    assert np.array_equal(adct.scale_vector(kind, n), M.scale_vector(kind, n))


@pytest.mark.parametrize("kind", M.KINDS)
@pytest.mark.parametrize("n", M.SIZES)
@pytest.mark.parametrize("qstep", (1, 8, 13, 16, 32, 64, 100, 4096))
def test_quant_tables(kind, n, qstep):
    mq, dq = adct.quant_tables(kind, n, qstep)
    omq, odq = P.quant_tables(kind, n, qstep)
    assert np.array_equal(mq, omq)
    assert np.array_equal(dq, odq)


def _compress(lib, **kw):
    args = dict(transform=1, n=8, r=10, qstep=0, src=C.c_void_p(4096), dtype=0, batch=1,
                height=64, width=64, pitch=64, stride=64 * 64, kept=None, scaled=None,
                recon=None, sse=None, stream=None)
    args.update(kw)
    return lib.adct_compress(args["transform"], args["n"], args["r"], args["qstep"], args["src"],
                             args["dtype"], args["batch"], args["height"], args["width"],
                             args["pitch"], args["stride"], args["kept"], args["scaled"],
                             args["recon"], args["sse"], args["stream"])


@pytest.mark.parametrize("kw,status", [
    (dict(transform=7), -1), (dict(transform=0), -1), (dict(transform=3, n=16), -1),
    (dict(transform=4, n=32), -1), (dict(n=4), -1), (dict(n=128), -1),
    (dict(n=64, dtype=1, pitch=64), -1), (dict(n=64, qstep=8), -1), (dict(n=64, transform=3), -1),
    (dict(r=0), -1), (dict(r=65), -1), (dict(n=16, r=257), -1), (dict(qstep=-1), -1),
    (dict(qstep=4097), -1), (dict(dtype=2), -1), (dict(src=None), -1),
    (dict(height=60), -2), (dict(width=20, pitch=20), -2), (dict(pitch=32), -2),
    (dict(batch=2, stride=100), -2), (dict(batch=-1), -2),
    (dict(src=C.c_void_p(4097)), -3), (dict(pitch=68), -3), (dict(n=16, pitch=72), -3),
    (dict(dtype=1, pitch=68), -3), (dict(sse=C.c_void_p(4100)), -3),
])
def test_argument_errors_are_reported_before_launch(lib, kw, status):
    assert _compress(lib, **kw) == status
    assert lib.adct_last_error()


def test_empty_image_sets_are_a_no_op(lib):
    # empty tensors carry null pointers; nothing is launched
    assert _compress(lib, batch=0, src=None) == 0
    assert _compress(lib, height=0, src=None) == 0
    assert lib.adct_fwd2d(1, 16, None, 0, 0, 16, 16, 16, 256, None, None) == 0
    assert lib.adct_decompress(2, 8, 5, 0, None, None, 1, 1, 0, 8, 8, 0, None) == 0


def test_mfma_entry_point_validates(lib):
    p = C.c_void_p(4096)
    #                              T  r   src  B  H   W   pitch stride kept scaled recon sse
    assert lib.adct_compress_mfma(7, 10, p, 1, 64, 64, 64, 4096, None, None, None, None, None) == -1
    assert lib.adct_compress_mfma(1, 0, p, 1, 64, 64, 64, 4096, None, None, None, None, None) == -1
    assert lib.adct_compress_mfma(1, 65, p, 1, 64, 64, 64, 4096, None, None, None, None, None) == -1
    assert lib.adct_compress_mfma(1, 10, None, 1, 64, 64, 64, 4096, None, None, None, None,
                                  None) == -1
    assert lib.adct_compress_mfma(1, 10, p, 1, 60, 64, 64, 4096, None, None, None, None, None) == -2
    assert lib.adct_compress_mfma(1, 10, p, 1, 64, 64, 68, 4096, None, None, None, None, None) == -3
    assert lib.adct_compress_mfma(1, 10, p, 1, 64, 64, 64, 4096, None, None, C.c_void_p(4100),
                                  None, None) == -3
    assert lib.adct_compress_mfma(1, 10, None, 0, 64, 64, 64, 4096, None, None, None, None,
                                  None) == 0


def test_other_entry_points_validate(lib):
    p = C.c_void_p(4096)
    assert lib.adct_fwd2d(1, 8, None, 0, 1, 8, 8, 8, 64, p, None) == -1
    assert lib.adct_fwd2d(1, 8, p, 0, 1, 8, 8, 8, 64, C.c_void_p(4100), None) == -3
    assert lib.adct_inv2d(1, 8, 0, 0, p, p, 0, 1, 8, 8, 8, 64, None) == -1
    assert lib.adct_inv2d(2, 16, 10, 0, p, p, 0, 1, 24, 16, 16, 384, None) == -2
    assert lib.adct_decompress(1, 32, 10, 0, None, p, 0, 1, 32, 32, 32, 1024, None) == -1
    assert lib.adct_get_matrix(1, 12, 0, p) == -1
    assert lib.adct_zigzag(7, p) == -1
    assert lib.adct_quant_tables(1, 8, 0, p, p) == -1
    # streaming ceilings: patterns 0-5, 16-byte multiples, a source unless writing
    assert lib.adct_stream_ceiling(6, p, p, 16, 1, 1, None) == -1
    assert lib.adct_stream_ceiling(2, p, p, 24, 1, 1, None) == -1
    assert lib.adct_stream_ceiling(5, p, None, 16, 1, 1, None) == -1
    assert lib.adct_stream_ceiling(3, p, p, 16, 1, 3, None) == -1
    assert lib.adct_stream_ceiling(4, p, None, 0, 1, 1, None) == 0     # nothing to write


def test_quality_entry_points_validate(lib):
    p = C.c_void_p(4096)
    # psnr: negative count, zero pixels, null and misaligned buffers; count 0 is a no-op
    assert lib.adct_psnr(-1, 64, p, p, None) == -1
    assert lib.adct_psnr(3, 0, p, p, None) == -1
    assert lib.adct_psnr(3, 64, None, p, None) == -1
    assert lib.adct_psnr(3, 64, C.c_void_p(4100), p, None) == -3
    assert lib.adct_psnr(0, 64, None, None, None) == 0
    # moments: transform, n, shape, record alignment, more than 2^32 tiles is refused
    assert lib.adct_moments(7, 8, p, 0, 1, 8, 8, 8, 64, p, None) == -1
    assert lib.adct_moments(3, 16, p, 0, 1, 16, 16, 16, 256, p, None) == -1
    assert lib.adct_moments(1, 12, p, 0, 1, 12, 12, 12, 144, p, None) == -1
    assert lib.adct_moments(1, 8, p, 0, 1, 12, 8, 8, 96, p, None) == -2
    assert lib.adct_moments(1, 8, p, 0, 1, 8, 8, 8, 64, C.c_void_p(4100), None) == -3
    assert lib.adct_moments(1, 8, p, 0, 1, 8, 8, 8, 64, None, None) == -1
    assert lib.adct_moments(1, 8, p, 0, 0, 8, 8, 8, 64, None, None) == 0
    assert lib.adct_moments(1, 8, p, 0, 1, 1 << 19, 1 << 19, 1 << 19, 1 << 38, p, None) == -2
    # coding gains: basis, counts, null pointers
    assert lib.adct_coding_gain(1, 8, 2, 1, p, p, None) == -1
    assert lib.adct_coding_gain(1, 8, 1, -1, p, p, None) == -1
    assert lib.adct_coding_gain(1, 8, 1, 1, None, p, None) == -1
    assert lib.adct_coding_gain(1, 8, 1, 0, None, None, None) == 0
    assert lib.adct_coding_gain_ar1(2, 16, 5, 1, p, p, p, None) == -1
    assert lib.adct_coding_gain_ar1(2, 16, 0, 1, None, p, p, None) == -1
    assert lib.adct_coding_gain_ar1(2, 16, 0, 4, p, None, None, None) == 0
    assert lib.adct_coding_gain_ar1(2, 16, 0, 4, C.c_void_p(4098), p, None, None) == -3


def test_dct_entry_points_validate(lib):
    # the exact DCT (float32) is 8-point, zonal, without integer coefficients
    p = C.c_void_p(4096)
    out = np.zeros(64, dtype=np.int32)
    assert lib.adct_get_matrix(6, 8, 0, out.ctypes.data) == -1
    assert lib.adct_quant_tables(6, 8, 16, out.ctypes.data, out.ctypes.data) == -1
    assert np.array_equal(adct.scale_vector(6, 8), np.ones(8))
    assert _compress(lib, transform=6, kept=p) == -1
    assert _compress(lib, transform=6, qstep=8) == -1
    assert _compress(lib, transform=6, n=16, pitch=64) == -1
    assert lib.adct_fwd2d(6, 8, p, 0, 1, 8, 8, 8, 64, p, None) == -1
    assert lib.adct_inv2d(6, 8, 10, 0, p, p, 0, 1, 8, 8, 8, 64, None) == -1
    assert lib.adct_moments(6, 8, p, 0, 1, 8, 8, 8, 64, p, None) == -1
    assert lib.adct_coding_gain_ar1(6, 8, 1, 1, p, p, None, None) == -1
    assert lib.adct_compress_mfma(6, 10, p, 1, 64, 64, 64, 4096, None, None, None, None, None) == -1


def test_python_front_end_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    x = torch.zeros((8, 8), dtype=torch.uint8)
    with pytest.raises(ValueError):
        adct.compress(x, 1, 8, 10)
    with pytest.raises(ValueError):
        adct.fwd2d(x, 1, 8)


def test_batch_plan_validation_before_gpu(lib):
    import numpy as np
    descs = np.zeros(1, dtype=adct.IMAGE_DESC)
    descs[0] = (0, 0, 64, 64, 64, 1, 10, 0)
    tus = np.zeros(1, dtype=adct.TU_DESC)
    tus[0] = (0, 0, 0, 8)
    h = C.c_void_p()
    w = C.c_int64()

    def create(d, t, dtype=0):
        return lib.adct_batch_create(d.ctypes.data, len(d), t.ctypes.data, len(t), dtype,
                                     None, C.byref(w), C.byref(h))

    bad = tus.copy(); bad[0] = (0, 60, 0, 8)        # outside the image
    assert create(descs, bad) == -2
    bad[0] = (0, 8, 0, 16)                          # not aligned to its size
    assert create(descs, bad) == -2
    bad[0] = (1, 0, 0, 8)                           # no such image
    assert create(descs, bad) == -2
    bad[0] = (0, 0, 0, 12)                          # bad size
    assert create(descs, bad) == -2
    d2 = descs.copy(); d2[0]["height"] = 60         # not a multiple of 8
    assert create(d2, tus) == -2
    d2 = descs.copy(); d2[0]["transform"] = 3
    assert create(d2, tus) == -1
    d2 = descs.copy(); d2[0]["src_offset"] = 4      # not 16-byte aligned
    assert create(d2, tus) == -3
    assert create(descs, tus, dtype=5) == -1
    two = np.zeros(2, dtype=adct.TU_DESC)
    two[0], two[1] = (0, 0, 0, 16), (0, 8, 8, 8)    # the 8x8 TU lies inside the 16x16 one
    assert create(descs, two) == -2
    assert "overlaps" in lib.adct_last_error().decode()
    two[1] = (0, 16, 0, 8)                          # neighbours: validation passes
    st = create(descs, two)
    assert st in (0, -4)                            # -4: no device to build the plan on
    if st == 0:
        lib.adct_batch_destroy(h)
    assert lib.adct_batch_run(None, None, None, None, None, None, None, 0, None) == -1


def test_product_path_never_touches_the_oracle():
    # the package and its native sources name neither the oracle package nor
    # any fallback to it; only tests, smoke() and the bench's CPU leg may
    import ast
    import pathlib
    pkg = pathlib.Path(__file__).resolve().parents[1] / "paper_2207_11638_amd"
    for path in pkg.rglob("*.py"):
        tree = ast.parse(path.read_text())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            else:
                continue
            assert not any(n == "oracle" or n.startswith("oracle.") for n in names), path
    for path in (pkg / "csrc").iterdir():
        assert "oracle" not in path.read_text().lower(), path


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    from paper_2207_11638_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing" / "libadct.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L.load()


@pytest.mark.parametrize("kind,n", [(k, n) for k in M.KINDS for n in M.SIZES] +
                         [(k, 8) for k in M.COMPARISON_KINDS])
def test_transform_measures_match_the_oracle(kind, n):
    from oracle import metrics as Q
    eps, delta = adct.transform_measures(kind, n)
    want_eps = Q.total_error_energy(M.dct2_matrix(n), M.near_orthogonal(kind, n))
    t = M.transform_matrix(kind, n)
    want_delta = Q.deviation_from_diagonality(t @ t.T)
    assert eps == pytest.approx(want_eps, rel=1e-12, abs=1e-12)
    assert delta == pytest.approx(want_delta, rel=1e-12, abs=1e-15)


def test_transform_measures_reproduce_table1(paper_values):
    v = paper_values["total_error_energy"]
    assert round(adct.transform_measures(M.ROUND, 8)[0], 2) == v["round_8"]
    assert round(adct.transform_measures(M.SIGN, 8)[0], 2) == v["sign_8"]
    assert round(adct.transform_measures(M.SDCT, 8)[0], 2) == v["sdct_8"]
    assert round(adct.transform_measures(M.WHT, 8)[0], 2) == 5.05
    assert round(adct.transform_measures(M.HT, 8)[0], 2) == 47.61
    assert adct.transform_measures(M.SIGN, 8)[1] == pytest.approx(1 / 14, abs=1e-15)
    assert adct.transform_measures(M.ROUND, 8)[1] == pytest.approx(4 / 69, abs=1e-15)
    assert adct.transform_measures(6, 8) == (0.0, 0.0)
