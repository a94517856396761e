"""GPU parity of the serving engine: every request of a mixed batch against
the oracle, a request alone against the same request inside a mix, many
batches through a small arena (admission waits and ring wrap-around), more
than 64 requests per class launch, and a real-time trace replay."""
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

DEV = torch.device("cuda:0")


def stream():
    return torch.cuda.current_stream().cuda_stream


class Job:
    """One request: its image on the GPU (optionally with padded rows) and
    pinned host buffers that receive its outputs."""

    def __init__(self, tag, h, w, n, kind, r, q=0, dtype="u8", scaled=False, pad=0, seed=0):
        self.tag, self.h, self.w, self.n, self.kind, self.r, self.q = tag, h, w, n, kind, r, q
        self.scaled = scaled
        if dtype == "u8":
            self.img = synth.ar1_image(h, w, rho=0.9, seed=seed)
        else:
            self.img = synth.laplace_residual(h, w, seed=seed)
        pitch = w + pad
        full = np.zeros((h, pitch), dtype=self.img.dtype)
        full[:, :w] = self.img
        self.full = torch.from_numpy(full).to(DEV)
        self.x = self.full[:, :w]
        tiles = (h // n) * (w // n)
        self.h_kept = torch.empty(tiles * r, dtype=torch.int32).pin_memory()
        self.h_scaled = torch.empty(tiles * r, dtype=torch.float32).pin_memory() if scaled else None
        self.h_recon = torch.empty((h, pitch), dtype=self.full.dtype).pin_memory()
        self.rec = adct.request(self.x, kind, n, r, q, tag=tag, want_scaled=scaled,
                                h_kept=self.h_kept, h_scaled=self.h_scaled, h_recon=self.h_recon)

    def outputs(self):
        th, tw = self.h // self.n, self.w // self.n
        out = {"kept": self.h_kept.numpy().reshape(th, tw, self.r),
               "recon": self.h_recon.numpy()[:, : self.w]}
        if self.scaled:
            out["scaled"] = self.h_scaled.numpy().reshape(th, tw, self.r)
        return out

    def check(self, sse):
        want = P.compress(self.img, self.kind, self.n, self.r, self.q)
        got = self.outputs()
        ctx = f"tag={self.tag} {self.h}x{self.w} n={self.n} T{self.kind} r={self.r} q={self.q}"
        assert np.array_equal(got["kept"], want["kept"]), ctx
        assert np.array_equal(got["recon"], want["recon"]), ctx
        assert int(sse) == want["sse"], ctx
        if self.scaled:
            s, w = got["scaled"].astype(np.float64), want["scaled"]
            nz = w != 0
            assert np.all(s[~nz] == 0), ctx
            assert np.all(np.abs(s[nz] - w[nz]) <= 1e-5 * np.abs(w[nz])), ctx


def mixed_jobs(seed, count=24, tag0=0):
    rng = synth.rng_for(seed)
    sizes = [(64, 64), (96, 160), (32, 224), (128, 96), (160, 32), (32, 32), (224, 128)]
    jobs = []
    for i in range(count):
        h, w = sizes[i % len(sizes)]
        n = (8, 16, 32)[i % 3]
        dtype = "u8" if i % 4 else "i16"
        q = 0 if i % 5 else (8, 16, 64)[i % 3]
        r = [1, 6, 10, 28, n * n, 45 if n > 8 else 64][int(rng.integers(0, 6))]
        r = min(r, n * n)
        jobs.append(Job(tag0 + i, h, w, n, 1 + (i // 3) % 2, r, q, dtype,
                        scaled=bool(i % 2), pad=32 * (i % 3 == 1), seed=seed * 100 + i))
    return jobs


def serve_all(jobs, budget=1 << 28, max_inflight=2, max_batch=256):
    """Submit every job (flushing and polling while the budget is full),
    drain, and return {tag: completion} plus the server's statistics."""
    srv = adct.Server(budget, max_inflight=max_inflight, max_batch=max_batch, stream=stream())
    done = {}
    pending = list(jobs)
    while pending:
        if srv.submit(pending[0].rec):
            pending.pop(0)
            continue
        srv.flush()
        for c in srv.poll(wait=True):
            done[int(c["tag"])] = c
    while srv.flush():
        pass
    while len(done) < len(jobs):
        got = srv.poll(wait=True)
        for c in got:
            done[int(c["tag"])] = c
        srv.flush()
        assert len(got) or srv.stats()["in_flight"] or srv.stats()["queued"]
    stats = srv.stats()
    srv.close()
    return done, stats


def test_mixed_batch_matches_oracle():
    jobs = mixed_jobs(seed=11)
    srv = adct.Server(1 << 28, max_inflight=2, max_batch=64, stream=stream())
    for j in jobs:
        assert srv.submit(j.rec)
    assert srv.flush() == len(jobs)
    done = srv.poll(wait=True)
    assert len(done) == len(jobs)
    assert set(done["batch"].tolist()) == {0}
    for c in done:
        jobs[int(c["tag"])].check(c["sse"])
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["in_flight"] == 0 and st["batches"] == 1
    srv.close()


def test_alone_equals_in_mix():
    probe_a = Job(100, 96, 160, 16, 2, 28, 0, "u8", scaled=True, seed=7)
    probe_b = Job(100, 96, 160, 16, 2, 28, 0, "u8", scaled=True, seed=7)
    alone, _ = serve_all([probe_a])
    mix = mixed_jobs(seed=12, count=12)
    mixed, _ = serve_all(mix[:6] + [probe_b] + mix[6:])
    a, b = probe_a.outputs(), probe_b.outputs()
    for key in ("kept", "recon", "scaled"):
        assert np.array_equal(a[key], b[key]), key
    assert int(alone[100]["sse"]) == int(mixed[100]["sse"])
    probe_a.check(alone[100]["sse"])


def test_many_batches_through_a_small_arena():
    jobs = mixed_jobs(seed=13, count=30)
    # room for a few requests at a time: admission waits and the ring wraps
    budget = 3 * max(j.h * j.full.shape[1] * j.full.element_size() * 2 + j.h_kept.numel() * 8
                     + 4096 for j in jobs)
    done, stats = serve_all(jobs, budget=budget, max_inflight=2, max_batch=4)
    assert stats["refused"] > 0 and stats["batches"] >= 8
    assert stats["charged"] >= 0 and stats["completed"] == len(jobs)
    for j in jobs:
        j.check(done[j.tag]["sse"])


def test_more_than_64_requests_per_class_launch():
    jobs = [Job(i, 64, 64, 8, 1, 10, seed=500 + i) for i in range(150)]
    jobs += [Job(150 + i, 32, 64, 16, 2, 28, seed=700 + i) for i in range(90)]
    srv = adct.Server(1 << 28, max_inflight=1, max_batch=256, stream=stream())
    for j in jobs:
        assert srv.submit(j.rec)
    assert srv.flush() == len(jobs)
    done = srv.poll(wait=True)
    assert len(done) == len(jobs)
    for c in done:
        jobs[int(c["tag"])].check(c["sse"])
    srv.close()


def test_trace_replay():
    rng = synth.rng_for(21)
    jobs = []
    for i in range(160):
        n = (8, 16, 32)[int(rng.integers(0, 3))]
        h, w = (int(v) * 32 for v in rng.integers(1, 8, size=2))
        jobs.append(Job(i, h, w, n, 1 + int(rng.integers(0, 2)), int(rng.integers(6, 29)),
                        seed=900 + i))
    arrival_ms = synth.poisson_arrivals(len(jobs), rate_hz=20000.0, seed=22) * 1e3
    reqs = np.stack([j.rec for j in jobs])
    srv = adct.Server(1 << 22, max_inflight=2, max_batch=64, stream=stream())
    lat, batch, sse = srv.run_trace(reqs, arrival_ms)
    st = srv.stats()
    srv.close()
    assert np.all(np.isfinite(lat)) and np.all(lat > 0)
    assert np.all(np.diff(batch) >= 0)          # first come, first served
    assert st["completed"] == len(jobs) and st["queued"] == 0 and st["in_flight"] == 0
    for j in jobs:
        want = P.compress(j.img, j.kind, j.n, j.r, 0)
        got = j.outputs()
        assert np.array_equal(got["kept"], want["kept"]), j.tag
        assert np.array_equal(got["recon"], want["recon"]), j.tag
        assert int(sse[j.tag]) == want["sse"], j.tag
