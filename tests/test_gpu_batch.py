"""GPU parity of the ragged batch path: every TU of a mixed 8/16/32 quadtree
batch against the oracle applied to that block, and the three run modes
(one launch per bucket, graph replay, one launch per image) against each
other."""
import math

import numpy as np
import pytest

from oracle import pipeline as P
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2207_11638_amd as adct  # noqa: E402
from paper_2207_11638_amd import ragged  # noqa: E402

DEV = torch.device("cuda:0")


def make_set(kind, seed, n_images=7, r_set=(1, 6, 10, 28, 45, 64, 1024)):
    rng = synth.rng_for(seed)
    sizes = [(64, 96), (40, 72), (96, 64), (8, 8), (136, 200), (32, 40), (72, 104)][:n_images]
    imgs, tus, kinds, rs, qs = [], [], [], [], []
    for i, (h, w) in enumerate(sizes):
        if kind == "u8":
            imgs.append(synth.ar1_image(h, w, rho=0.9, seed=seed + i))
        else:
            imgs.append(synth.laplace_residual(h, w, seed=seed + i))
        tus.append(synth.quadtree_tus(h, w, rng, p_split=0.4))
        kinds.append(1 + i % 2)
        rs.append(r_set[i % len(r_set)])
        qs.append(0 if kind == "u8" or i % 3 == 0 else [8, 16, 64][i % 3])
    arena, descs = ragged.pack_images(imgs, kinds, rs, qs)
    return imgs, descs, ragged.tu_table(tus), arena


def oracle_expect(imgs, descs, tus):
    kept = {}
    recon = [np.zeros_like(im) for im in imgs]
    scaled = {}
    sse = [0] * len(imgs)
    for t, tu in enumerate(tus):
        i, x, y, n = int(tu["image"]), int(tu["x"]), int(tu["y"]), int(tu["n"])
        d = descs[i]
        r = min(int(d["r"]), n * n)
        out = P.compress(imgs[i][y:y + n, x:x + n], int(d["transform"]), n, r, int(d["qstep"]))
        kept[t] = out["kept"].reshape(-1)
        scaled[t] = out["scaled"].reshape(-1)
        recon[i][y:y + n, x:x + n] = out["recon"]
        sse[i] += out["sse"]
    return kept, scaled, recon, sse


def run_plan(plan, arena, mode, stream=None):
    src = torch.from_numpy(arena).to(DEV)
    dst = torch.zeros_like(src)
    kept = torch.zeros(max(1, plan.kept_words), dtype=torch.int32, device=DEV)
    scaled = torch.zeros(max(1, plan.kept_words), dtype=torch.float32, device=DEV)
    n = len(plan.images)
    sse = torch.full((n,), 7, dtype=torch.uint64, device=DEV)   # overwritten by the run
    psnr = torch.zeros(n, dtype=torch.float32, device=DEV)
    plan.run(src, dst, kept, scaled, sse, psnr, mode=mode)
    torch.cuda.synchronize()
    return (dst.cpu().numpy(), kept.cpu().numpy(), scaled.cpu().numpy(),
            sse.cpu().numpy().astype(np.int64), psnr.cpu().numpy())


# r_set: the default mixes kept bounds above 8 into the zonal class, so its
# unified launch is the general one; the second keeps every r <= 36 and
# selects the row-per-thread launch of small kept bounds
@pytest.mark.parametrize("r_set,small", [((1, 6, 10, 28, 45, 64, 1024), 0),
                                         ((1, 6, 10, 15, 21, 28, 36), 1)])
@pytest.mark.parametrize("mode", ["batched", "unified"])
@pytest.mark.parametrize("kind", ["u8", "i16"])
def test_batch_matches_oracle_per_tu(kind, mode, r_set, small):
    imgs, descs, tus, arena = make_set(kind, 5000 if kind == "u8" else 6000, r_set=r_set)
    plan = adct.BatchPlan(descs, tus, torch.uint8 if kind == "u8" else torch.int16)
    info = plan.info()
    assert info["tus"] == len(tus) and info["items8"] > 0 and info["items16"] > 0
    assert info["small_bound"] == small and info["unified_items"] > 0
    dst, kept, scaled, sse, psnr = run_plan(plan, arena, mode)
    want_kept, want_scaled, want_recon, want_sse = oracle_expect(imgs, descs, tus)
    for t in range(len(tus)):
        o = int(plan.tu_kept_offset[t])
        k = want_kept[t]
        assert np.array_equal(kept[o:o + len(k)], k), t
        ws = want_scaled[t]
        got = scaled[o:o + len(ws)].astype(np.float64)
        nz = ws != 0
        assert np.all(got[~nz] == 0)
        assert np.all(np.abs(got[nz] - ws[nz]) <= 1e-5 * np.abs(ws[nz]))
    for i, d in enumerate(descs):
        assert np.array_equal(ragged.unpack_image(dst, d), want_recon[i]), i
        assert sse[i] == want_sse[i]
        npix = int(d["height"]) * int(d["width"])
        want_p = math.inf if want_sse[i] == 0 else 10 * math.log10(65025.0 * npix / want_sse[i])
        if math.isinf(want_p):
            assert math.isinf(psnr[i])
        else:
            assert abs(psnr[i] - want_p) <= 1e-5 * want_p
    assert plan.kept_words == sum(len(v) for v in want_kept.values())


def test_run_modes_and_shapes_agree():
    imgs, descs, tus, arena = make_set("u8", 7000)
    plan = adct.BatchPlan(descs, tus, torch.uint8)
    base = run_plan(plan, arena, "batched")
    for mode in ("per_image", "batched", "unified"):
        got = run_plan(plan, arena, mode)
        for a, b in zip(base, got):
            assert np.array_equal(a, b)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(3):    # replays of one captured graph
            got = run_plan(plan, arena, "graph")
            for a, b in zip(base, got):
                assert np.array_equal(a, b)
    for bs8, bsj in ((64, 128), (256, 256), (64, 256)):
        plan.set_shape(bs8, bsj)
        got = run_plan(plan, arena, "batched")
        for a, b in zip(base, got):
            assert np.array_equal(a, b)


def test_tune_picks_a_valid_shape_and_keeps_results():
    imgs, descs, tus, arena = make_set("u8", 8000)
    plan = adct.BatchPlan(descs, tus, torch.uint8)
    base = run_plan(plan, arena, "batched")
    src = torch.from_numpy(arena).to(DEV)
    dst = torch.zeros_like(src)
    kept = torch.zeros(plan.kept_words, dtype=torch.int32, device=DEV)
    chosen = plan.tune(src, dst, kept)
    assert set(chosen.tolist()) <= {64, 128, 256}
    got = run_plan(plan, arena, "batched")
    for a, b in zip(base, got):
        assert np.array_equal(a, b)


def test_tune_cache_is_reused_by_a_second_plan(tmp_path, monkeypatch):
    """With ADCT_TUNE_CACHE set, a second plan over the same TUs finds every
    choice of the first plan's tuning in the cache (nothing is appended) and
    makes the same choices."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("ADCT_TUNE_CACHE", str(cache))
    imgs, descs, tus, arena = make_set("u8", 8100)
    src = torch.from_numpy(arena).to(DEV)
    dst = torch.zeros_like(src)
    plan = adct.BatchPlan(descs, tus, torch.uint8)
    kept = torch.zeros(plan.kept_words, dtype=torch.int32, device=DEV)
    chosen = plan.tune(src, dst, kept)
    lines = cache.read_text().splitlines()
    assert len(lines) >= len(chosen)
    again = adct.BatchPlan(descs, tus, torch.uint8)
    chosen2 = again.tune(src, dst, kept)
    assert cache.read_text().splitlines() == lines
    assert chosen2.tolist() == chosen.tolist()
    assert again.info() == plan.info()
    for a, b in zip(run_plan(plan, arena, "batched"), run_plan(again, arena, "batched")):
        assert np.array_equal(a, b)


def test_boundary_split_of_residual_frame():
    # 4:2:0 residual planes whose heights are not multiples of 32: CTUs of 32
    # with forced splits on the border only (the implicit split)
    rng = synth.rng_for(1)
    planes = synth.residual_frame_planes(0, luma_h=80, luma_w=96)
    tus = [synth.quadtree_tus(p.shape[0], p.shape[1], rng, p_split=0.0) for p in planes]
    assert any((t[:, 2] == 16).any() for t in tus)
    arena, descs = ragged.pack_images(planes, [2, 2, 2], [1024, 1024, 1024], [16, 16, 16])
    tut = ragged.tu_table(tus)
    plan = adct.BatchPlan(descs, tut, torch.int16)
    dst, kept, scaled, sse, psnr = run_plan(plan, arena, "batched")
    _, _, want_recon, want_sse = oracle_expect(planes, descs, tut)
    for i, d in enumerate(descs):
        assert np.array_equal(ragged.unpack_image(dst, d), want_recon[i])
        assert sse[i] == want_sse[i]


@pytest.mark.parametrize("shape", [(1, 1, False, 8), (4, 4, False, 8), (2, 2, True, 8),
                                   (1, 4, True, 4), (4, 1, True, 1)])
def test_small_bound_shapes_agree_with_the_oracle(shape):
    """Every shape of the row-per-thread unified launch (groups per item, the
    persistent grid) gives the oracle's outputs for every TU."""
    imgs, descs, tus, arena = make_set("u8", 9000, r_set=(1, 6, 10, 15, 21, 28, 36))
    plan = adct.BatchPlan(descs, tus, torch.uint8)
    plan.set_small_shape(*shape)
    info = plan.info()
    assert info["small_bound"] == 1
    assert (info["small_groups8"], info["small_groups16"], info["persistent"],
            info["wgs_per_cu"]) == (shape[0], shape[1], int(shape[2]), shape[3])
    dst, kept, scaled, sse, psnr = run_plan(plan, arena, "unified")
    want_kept, want_scaled, want_recon, want_sse = oracle_expect(imgs, descs, tus)
    for t in range(len(tus)):
        o = int(plan.tu_kept_offset[t])
        assert np.array_equal(kept[o:o + len(want_kept[t])], want_kept[t]), t
    for i, d in enumerate(descs):
        assert np.array_equal(ragged.unpack_image(dst, d), want_recon[i]), i
        assert sse[i] == want_sse[i]


def test_tune_searches_the_small_bound_shape():
    imgs, descs, tus, arena = make_set("u8", 9100, r_set=(1, 6, 10, 15, 21, 28, 36))
    plan = adct.BatchPlan(descs, tus, torch.uint8)
    base = run_plan(plan, arena, "unified")
    src = torch.from_numpy(arena).to(DEV)
    dst = torch.zeros_like(src)
    kept = torch.zeros(plan.kept_words, dtype=torch.int32, device=DEV)
    plan.tune(src, dst, kept)
    info = plan.info()
    assert info["small_groups8"] in (1, 2, 4) and info["small_groups16"] in (1, 2, 4)
    assert info["persistent"] in (0, 1) and info["wgs_per_cu"] in (4, 8)
    got = run_plan(plan, arena, "unified")
    for a, b in zip(base, got):
        assert np.array_equal(a, b)
    with pytest.raises(adct.AdctError):
        plan.set_small_shape(3, 2)
