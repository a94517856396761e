"""GPU parity at the full workload sizes, in the launch configurations the
benchmark times: sampled outputs checked one by one against the oracle (which
computes a single tile, TU or request in milliseconds), plus exact properties
checked on every image (the error energy of each image against its
reconstruction, recomputed from scratch)."""
from concurrent.futures import ThreadPoolExecutor

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
WORKERS = 16


def exact_sse(x, recon):
    """Per-image sum of squared differences, exact, on the GPU (chunked)."""
    out = []
    for i in range(0, x.shape[0], 32):
        d = recon[i:i + 32].to(torch.int64) - x[i:i + 32].to(torch.int64)
        out.append((d * d).flatten(1).sum(1))
    return torch.cat(out).cpu().numpy()


def check_scaled(got, want):
    got = got.astype(np.float64)
    nz = want != 0
    assert np.all(got[~nz] == 0)
    assert np.all(np.abs(got[nz] - want[nz]) <= 1e-5 * np.abs(want[nz]))


@pytest.fixture(scope="module")
def c1_images():
    # drawn on threads: this process already uses the GPU, so it never forks
    imgs, _ = synth.ar1_batch(1024, 2048, 2048, workers=WORKERS)
    return imgs


def c1_spread(r):
    # images interleaved by the fused 8x8 kernel's dispatch order for this r
    return 64 if r <= 16 else (16 if r <= 45 else 2)


def oracle_images(imgs, picks, kind, r):
    with ThreadPoolExecutor(len(picks)) as ex:
        return list(ex.map(lambda i: P.compress(imgs[i], kind, 8, r), picks))


@pytest.mark.parametrize("kind", (1, 2))
@pytest.mark.parametrize("r", (1, 6, 10, 16, 28, 45, 64))
def test_c1_full_size(c1_images, kind, r):
    # 1024 x 2048^2 uint8, N = 8: the launch the benchmark times.  Whole
    # images spread over the interleave blocks (first, last of the first
    # block, first of the second, last) against the oracle, sampled tiles
    # of the others, and every image's error energy against its own
    # reconstruction
    x = torch.from_numpy(c1_images).to(DEV)
    out = adct.compress(x, kind, 8, r)
    torch.cuda.synchronize()
    sse = out["sse"].cpu().numpy().astype(np.int64)
    assert np.array_equal(sse, exact_sse(x, out["recon"]))
    s = c1_spread(r)
    picks = sorted({0, s - 1, s, 1023})
    wants = oracle_images(c1_images, picks, kind, r)
    for i, want in zip(picks, wants):
        assert np.array_equal(out["kept"][i].cpu().numpy(), want["kept"]), i
        check_scaled(out["scaled"][i].cpu().numpy(), want["scaled"])
        assert np.array_equal(out["recon"][i].cpu().numpy(), want["recon"]), i
        assert sse[i] == want["sse"], i
    rng = synth.rng_for(100 + r + 1000 * kind)
    picks = np.stack([rng.integers(0, 1024, 100), rng.integers(0, 256, 100),
                      rng.integers(0, 256, 100)], axis=1)
    idx = torch.from_numpy(picks).to(DEV)
    kept = out["kept"][idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    scaled = out["scaled"][idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    for n_, (i, ty, tx) in enumerate(picks):
        block = c1_images[i, 8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8]
        want = P.compress(block, kind, 8, r)
        assert np.array_equal(kept[n_], want["kept"].reshape(-1)), (i, ty, tx)
        check_scaled(scaled[n_], want["scaled"].reshape(-1))
        rec = out["recon"][i, 8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8].cpu().numpy()
        assert np.array_equal(rec, want["recon"]), (i, ty, tx)
    if r == 64:
        # full retention reconstructs every image exactly
        assert torch.equal(out["recon"], x) and sse.sum() == 0
    del out, x
    torch.cuda.empty_cache()


def _frame(f):
    return synth.residual_frame_planes(f)


@pytest.fixture(scope="module")
def c2_planes():
    with ThreadPoolExecutor(WORKERS) as ex:
        return [p for fr in ex.map(_frame, range(64)) for p in fr]


@pytest.mark.parametrize("n,kind,q", [(32, 2, 16), (16, 1, 64)])
def test_c2_full_size_sampled_tus(c2_planes, n, kind, q):
    # 64 residual frames, every coefficient quantised, implicit split at the
    # 2160 / 1080 borders: the TU-list launch the benchmark times (tuned
    # per-bucket sequence)
    planes = c2_planes
    arena, descs = ragged.pack_images(planes, [kind] * len(planes), [n * n] * len(planes),
                                      [q] * len(planes))
    tus = ragged.tu_table([synth.quadtree_tus_fast(p.shape[0], p.shape[1], synth.rng_for(0),
                                                   p_split=0.0, ctu=n) for p in planes])
    plan = adct.BatchPlan(descs, tus, torch.int16)
    src = torch.from_numpy(arena).to(DEV)
    dst = torch.zeros_like(src)
    kept = torch.zeros(plan.kept_words, dtype=torch.int32, device=DEV)
    sse = torch.zeros(len(planes), dtype=torch.uint64, device=DEV)
    plan.tune(src, dst, kept, None, sse)
    plan.run(src, dst, kept, None, sse, mode="batched")
    torch.cuda.synchronize()
    sse_h = sse.cpu().numpy().astype(np.int64)
    dst_h, kept_h = dst.cpu().numpy(), kept.cpu().numpy()
    rng = synth.rng_for(7)
    for t in rng.choice(len(tus), size=300, replace=False):
        i, x0, y0, nn = (int(tus[t][f]) for f in ("image", "x", "y", "n"))
        want = P.compress(planes[i][y0:y0 + nn, x0:x0 + nn], kind, nn, nn * nn, q)
        o = int(plan.tu_kept_offset[t])
        assert np.array_equal(kept_h[o:o + nn * nn], want["kept"].reshape(-1)), t
        d = descs[i]
        p = int(d["pitch"])
        base = int(d["dst_offset"]) + y0 * p + x0
        rows = np.stack([dst_h[base + yy * p: base + yy * p + nn] for yy in range(nn)])
        assert np.array_equal(rows, want["recon"]), t
    for i in (0, 1, 2, len(planes) - 1):
        rec = ragged.unpack_image(dst_h, descs[i]).astype(np.int64)
        assert int(((rec - planes[i]) ** 2).sum()) == sse_h[i]


def test_c3_full_size_sampled_tus():
    # 10000 ragged images, quadtree TUs, graph replay of the tuned sequence
    n = 10000
    sizes = synth.ragged_sizes(n, seed=3000)
    hs, ws = sizes[:, 0], sizes[:, 1]
    rhos = np.array([synth.rng_for(1_003_000 + i).uniform(0.85, 0.98) for i in range(n)])
    pitches = (ws + 15) // 16 * 16
    offsets = np.zeros(n, dtype=np.int64)
    off = 0
    for i in range(n):
        off = (off + 255) // 256 * 256
        offsets[i] = off
        off += int(pitches[i] * hs[i])
    total = (off + 255) // 256 * 256
    arena = synth.ar1_arena(offsets, hs, ws, pitches, 3000 + np.arange(n), rhos, total,
                            workers=WORKERS)
    rs = synth.rng_for(3002).integers(6, 29, size=n)
    descs = np.zeros(n, dtype=adct.IMAGE_DESC)
    descs["src_offset"] = offsets
    descs["dst_offset"] = offsets
    descs["height"], descs["width"], descs["pitch"] = hs, ws, pitches
    descs["transform"] = 1 + np.arange(n) % 2
    descs["r"] = rs
    tus = ragged.tu_table([synth.quadtree_tus_fast(int(hs[i]), int(ws[i]),
                                                   synth.rng_for(4_000_000 + i))
                           for i in range(n)])
    plan = adct.BatchPlan(descs, tus, torch.uint8)
    src = torch.from_numpy(arena).to(DEV)
    dst = torch.zeros_like(src)
    kept = torch.zeros(plan.kept_words, dtype=torch.int32, device=DEV)
    sse = torch.zeros(n, dtype=torch.uint64, device=DEV)
    psnr = torch.zeros(n, dtype=torch.float32, device=DEV)
    plan.tune(src, dst, kept, None, sse)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(2):
            plan.run(src, dst, kept, None, sse, psnr, mode="graph")
    torch.cuda.synchronize()
    dst_h, kept_h = dst.cpu().numpy(), kept.cpu().numpy()
    sse_h = sse.cpu().numpy().astype(np.int64)
    rng = synth.rng_for(9)
    for t in rng.choice(len(tus), size=400, replace=False):
        i, x0, y0, nn = (int(tus[t][f]) for f in ("image", "x", "y", "n"))
        p = int(pitches[i])
        img = arena[int(offsets[i]):int(offsets[i]) + p * int(hs[i])].reshape(hs[i], p)
        r = min(int(rs[i]), nn * nn)
        want = P.compress(img[y0:y0 + nn, x0:x0 + nn], int(descs[i]["transform"]), nn, r)
        o = int(plan.tu_kept_offset[t])
        assert np.array_equal(kept_h[o:o + r], want["kept"].reshape(-1)), t
        rec = dst_h[int(offsets[i]):int(offsets[i]) + p * int(hs[i])].reshape(hs[i], p)
        assert np.array_equal(rec[y0:y0 + nn, x0:x0 + nn], want["recon"]), t
    for i in rng.choice(n, size=50, replace=False):
        p = int(pitches[i])
        a = arena[int(offsets[i]):int(offsets[i]) + p * int(hs[i])].reshape(hs[i], p)[:, :ws[i]]
        b = dst_h[int(offsets[i]):int(offsets[i]) + p * int(hs[i])].reshape(hs[i], p)[:, :ws[i]]
        d = a.astype(np.int64) - b.astype(np.int64)
        assert int((d * d).sum()) == sse_h[i], i


def test_c4_trace_at_full_rate_sampled_requests():
    # 2 s of the serving trace at 2000 requests/s (4000 requests, image sides
    # log-normal around 1024), 1 % of the requests checked against the oracle
    trace = synth.serving_requests(4000, seed=4000, rate_hz=2000.0)
    pool_n = 64
    sizes = np.array([(t["h"], t["w"]) for t in trace[:pool_n]], dtype=np.int64)
    px = sizes[:, 0] * sizes[:, 1]
    offsets = np.concatenate([[0], np.cumsum(px)[:-1]])
    arena = synth.ar1_arena(offsets, sizes[:, 0], sizes[:, 1], sizes[:, 1],
                            [5000 + i for i in range(pool_n)],
                            [0.85 + 0.13 * ((i * 0.618) % 1.0) for i in range(pool_n)],
                            int(px.sum()), workers=WORKERS)
    d_arena = torch.from_numpy(arena).to(DEV)
    pool = [d_arena[int(o):int(o) + int(p)].view(int(h), int(w))
            for o, p, (h, w) in zip(offsets, px, sizes)]
    recs, checks = [], []
    for i, t in enumerate(trace):
        j = i % pool_n
        h_kept = h_recon = None
        if i % 100 == 0:
            h, w = pool[j].shape
            h_kept = torch.empty((h // t["n"]) * (w // t["n"]) * t["r"],
                                 dtype=torch.int32).pin_memory()
            h_recon = torch.empty((h, w), dtype=torch.uint8).pin_memory()
            checks.append((i, j, h_kept, h_recon))
        recs.append(adct.request(pool[j], t["transform"], t["n"], t["r"], 0, tag=i,
                                 h_kept=h_kept, h_recon=h_recon))
    srv = adct.Server(32 << 30, max_inflight=2, max_batch=1024,
                      stream=torch.cuda.current_stream().cuda_stream)
    lat, batch, sse = srv.run_trace(np.stack(recs), np.array([t["t"] for t in trace]) * 1e3)
    srv.close()
    assert np.all(np.isfinite(lat)) and np.all(lat > 0) and np.all(np.diff(batch) >= 0)
    for i, j, hk, hr in checks:
        t = trace[i]
        img = arena[int(offsets[j]):int(offsets[j] + px[j])].reshape(int(sizes[j, 0]),
                                                                      int(sizes[j, 1]))
        want = P.compress(img, t["transform"], t["n"], t["r"])
        assert np.array_equal(hk.numpy().reshape(want["kept"].shape), want["kept"]), i
        assert np.array_equal(hr.numpy(), want["recon"]), i
        assert int(sse[i]) == want["sse"], i
