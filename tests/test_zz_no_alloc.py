"""The allocation-free entry point adct_compress_quality_noalloc against
adct_compress_quality (the same pipeline with a caller workspace), through
the C ABI: two calls in a row, the second on a smaller image set, so that
the shared scratch array is reused and must be cleared by each call."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU-only runs deselect these
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2207_11638_amd import _lib  # noqa: E402

DEV = torch.device("cuda:0")
SCRATCH_WORDS = 1 << 19


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def run(lib, noalloc, x, kind, n, r, q, with_cg):
    b, h, w = x.shape
    tiles = b * (h // n) * (w // n)
    kept = torch.full((tiles * r,), -7, dtype=torch.int32, device=DEV)
    scaled = torch.full((tiles * r,), -7.0, dtype=torch.float32, device=DEV)
    recon = torch.empty_like(x)
    psnr = torch.full((b,), -1.0, dtype=torch.float32, device=DEV)
    cg = torch.full((b,), -1.0, dtype=torch.float32, device=DEV) if with_cg else None
    dt = 0 if x.dtype == torch.uint8 else 1
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [kind, n, r, q, _p(x), dt, b, h, w, w, h * w, _p(kept), _p(scaled), _p(recon),
            _p(psnr), _p(cg), 1]
    if noalloc:
        status = lib.adct_compress_quality_noalloc(*args, stream)
    else:
        nbytes = lib.adct_compress_quality_workspace(n, b, int(with_cg))
        work = torch.empty(nbytes // 8, dtype=torch.uint64, device=DEV)
        status = lib.adct_compress_quality(*args, _p(work), nbytes, stream)
    assert status == 0, lib.adct_last_error()
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (kept, scaled, recon, psnr) + ((cg,) if with_cg else ())]


@pytest.mark.parametrize("kind,n,dtype,r,q", [(2, 8, "u8", 10, 0), (1, 16, "u8", 28, 0),
                                              (2, 32, "i16", 1024, 16)])
def test_noalloc_matches_workspace_entry_point(kind, n, dtype, r, q):
    lib = _lib.load()
    for i, (b, h, w) in enumerate(((3, 8 * n, 40 * n), (1, 4 * n, 9 * n))):
        if dtype == "u8":
            imgs = [synth.ar1_image(h, w, rho=0.93, seed=4000 + 10 * i + j) for j in range(b)]
        else:
            imgs = [synth.laplace_residual(h, w, seed=4100 + 10 * i + j) for j in range(b)]
        x = torch.from_numpy(np.stack(imgs)).to(DEV)
        want = run(lib, False, x, kind, n, r, q, True)
        got = run(lib, True, x, kind, n, r, q, True)
        for a, e in zip(got, want):
            assert np.array_equal(a, e)
        assert np.all(np.isfinite(got[3])) and np.all(np.isfinite(got[4]))


def test_noalloc_rejects_sets_beyond_the_scratch_array():
    lib = _lib.load()
    x = torch.zeros((1, 8, 8), dtype=torch.uint8, device=DEV)
    psnr = torch.zeros(1, dtype=torch.float32, device=DEV)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # batch * (1 + 3 * 64 + 4) words > 2^19: refused before any launch
    b = SCRATCH_WORDS // 197 + 1
    status = lib.adct_compress_quality_noalloc(1, 8, 10, 0, _p(x), 0, b, 8, 8, 8, 64, None, None,
                                               None, _p(psnr), _p(psnr), 1, stream)
    assert status == -5
    assert b"scratch" in lib.adct_last_error() or b"words" in lib.adct_last_error()
