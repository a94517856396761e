"""Seeded synthetic workload generators.

This module is shared by the tests, the benchmark and the oracle's callers.  It
draws random inputs only: images, residual frames, transform-unit layouts,
request traces.  It contains none of the transform arithmetic, so neither the
HIP library nor the oracle depends on the other through it.

Workloads (all seeded with NumPy's PCG64):

* 2D separable first-order Markov (AR(1)) images.  The paper models images as
  a first-order Markov process with covariance rho^|m-n| (section 4.1, coding
  gain); its 30 test images (section 5.1) are not available, so this field
  stands in for them.
* Laplacian prediction residuals (int16) with 4:2:0 chroma planes, standing in
  for the video sequences of section 6.2.
* HEVC-style quadtree partitions of an image into 8/16/32 transform units.
* Log-normal image sizes and Poisson arrival traces for the batched and
  served forms.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import lfilter

__all__ = [
    "rng_for",
    "ar1_field",
    "ar1_image",
    "ar1_batch_image",
    "ar1_batch",
    "laplace_residual",
    "residual_frame_planes",
    "quadtree_tus",
    "quadtree_tus_fast",
    "ar1_arena",
    "ar1_arena_image",
    "ragged_sizes",
    "poisson_arrivals",
    "serving_requests",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _round_half_away(x: np.ndarray) -> np.ndarray:
    # data quantisation of the synthetic field to integer grey levels
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def _ar1_along_rows(w: np.ndarray, rho: float) -> np.ndarray:
    """Stationary unit-variance AR(1) recursion along each row (axis 1).

    y[0] = w[0];  y[n] = rho*y[n-1] + sqrt(1-rho^2)*w[n].
    """
    c = np.sqrt(1.0 - rho * rho)
    w = np.array(w, dtype=np.float64, copy=True)
    # scale the first sample so that the filter output starts at y[0] = w[0]
    w[:, 0] /= c
    return lfilter([c], [1.0, -rho], w, axis=1)


def _ar1_along_columns(w: np.ndarray, rho: float) -> np.ndarray:
    """The same recursion down the columns (axis 0): y[0] = w[0] exactly, then
    the filter runs over rows 1.. with its state started at rho*y[0].  It is
    evaluated on the transposed field so that the filter walks contiguous
    memory; the arithmetic per sample is the recursion's own
    (rho*y[n-1] + c*w[n]), so the result does not depend on the layout."""
    c = np.sqrt(1.0 - rho * rho)
    wt = np.ascontiguousarray(w.T)
    yt = np.empty_like(wt)
    yt[:, 0] = wt[:, 0]
    if wt.shape[1] > 1:
        yt[:, 1:], _ = lfilter([c], [1.0, -rho], wt[:, 1:], axis=1,
                               zi=(rho * wt[:, 0])[:, None])
    return yt.T


def _to_u8(y: np.ndarray, sigma: float, mean: float) -> np.ndarray:
    """clip(round(mean + sigma*y), 0, 255) as uint8, with round half away from
    zero.  Every value that survives the clip is >= 0, where that rounding is
    floor(t + 1/2); negative values clip to 0 either way."""
    t = y * sigma
    t += mean
    t += 0.5
    np.floor(t, out=t)
    np.clip(t, 0, 255, out=t)
    return t.astype(np.uint8, order="C")   # row-major whatever the filter's layout


def ar1_field(h: int, w: int, rho: float, rng: np.random.Generator) -> np.ndarray:
    """Unit-variance 2D separable AR(1) Gaussian field (float64, h x w)."""
    white = rng.standard_normal((h, w))
    y = _ar1_along_rows(white, rho)
    return _ar1_along_columns(y, rho)


def ar1_image(h: int, w: int, rho: float = 0.95, sigma: float = 40.0,
              mean: float = 128.0, seed: int = 0) -> np.ndarray:
    """uint8 image: clip(round(mean + sigma*field), 0, 255)."""
    rng = rng_for(seed)
    return _to_u8(ar1_field(h, w, rho, rng), sigma, mean)


def ar1_batch_image(i: int, h: int, w: int, seed_base: int = 1000,
                    rho_lo: float = 0.85, rho_hi: float = 0.98,
                    sigma: float = 40.0, mean: float = 128.0):
    """Image ``i`` of a batch whose per-image rho ~ U[rho_lo, rho_hi].

    Both rho and the content come from seed ``seed_base + i``.  Returns
    ``(image_uint8, rho)``.
    """
    rng = rng_for(seed_base + i)
    rho = float(rng.uniform(rho_lo, rho_hi))
    return _to_u8(ar1_field(h, w, rho, rng), sigma, mean), rho


def ar1_batch(n: int, h: int, w: int, workers: int = 1, **kw):
    """Images 0..n-1 of ``ar1_batch_image`` as one (n, h, w) uint8 array.

    With ``workers`` > 1 the images are drawn by that many threads (NumPy and
    SciPy release the interpreter lock in the heavy steps); no process is
    forked, so this is safe in a process that already uses the GPU.  The
    content does not depend on the worker count.  Returns ``(images, rhos)``.
    """
    imgs = np.empty((n, h, w), dtype=np.uint8)
    rhos = np.zeros(n)

    def one(i):
        imgs[i], rhos[i] = ar1_batch_image(i, h, w, **kw)

    _run_threads(one, range(n), workers)
    return imgs, rhos


def _run_threads(fn, items, workers: int):
    """fn(item) for every item, on ``workers`` threads (in order when 1)."""
    items = list(items)
    if workers <= 1 or len(items) < 2:
        for it in items:
            fn(it)
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for _ in ex.map(fn, items):
            pass


def laplace_residual(h: int, w: int, scale: float = 12.0, clip: int = 255,
                     seed: int = 0) -> np.ndarray:
    """int16 i.i.d. Laplacian residual, rounded and clipped to [-clip, clip]."""
    rng = rng_for(seed)
    x = _round_half_away(rng.laplace(0.0, scale, size=(h, w)))
    return np.clip(x, -clip, clip).astype(np.int16)


def residual_frame_planes(frame: int, luma_h: int = 2160, luma_w: int = 3840,
                          scale: float = 12.0, seed_base: int = 2000):
    """One 4:2:0 residual frame: (Y, Cb, Cr) int16 planes.

    Plane p of frame f uses seed ``seed_base + 3*f + p``.
    """
    planes = []
    for p, (h, w) in enumerate([(luma_h, luma_w), (luma_h // 2, luma_w // 2),
                                (luma_h // 2, luma_w // 2)]):
        planes.append(laplace_residual(h, w, scale, 255, seed_base + 3 * frame + p))
    return planes


def quadtree_tus(h: int, w: int, rng: np.random.Generator, p_split: float = 0.4,
                 ctu: int = 32, min_tu: int = 8) -> np.ndarray:
    """HEVC-style quadtree partition of an h x w image into square TUs.

    The image is covered by ctu x ctu coding-tree units.  Each unit splits into
    four children with probability ``p_split`` per level down to ``min_tu``;
    a unit that crosses the image border is always split (implicit split).
    ``h`` and ``w`` must be multiples of ``min_tu``.

    Returns an int32 array of rows ``(x, y, size)`` in raster CTU order.
    """
    assert h % min_tu == 0 and w % min_tu == 0
    out = []

    def visit(x, y, s):
        if x >= w or y >= h:
            return
        inside = (x + s <= w) and (y + s <= h)
        if s > min_tu and (not inside or rng.random() < p_split):
            hs = s // 2
            visit(x, y, hs)
            visit(x + hs, y, hs)
            visit(x, y + hs, hs)
            visit(x + hs, y + hs, hs)
        else:
            out.append((x, y, s))

    for cy in range(0, h, ctu):
        for cx in range(0, w, ctu):
            visit(cx, cy, ctu)
    return np.asarray(out, dtype=np.int32).reshape(-1, 3)


def quadtree_tus_fast(h: int, w: int, rng: np.random.Generator, p_split: float = 0.4,
                      ctu: int = 32, min_tu: int = 8) -> np.ndarray:
    """Vectorised form of ``quadtree_tus`` (same model, different draw order):
    level by level, every block that lies inside the image splits with
    probability ``p_split`` and every block crossing the border splits; blocks
    entirely outside are dropped.  Returns int32 rows (x, y, size)."""
    assert h % min_tu == 0 and w % min_tu == 0
    ys, xs = np.meshgrid(np.arange(0, h, ctu), np.arange(0, w, ctu), indexing="ij")
    blocks = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int64)
    size = ctu
    out = []
    while len(blocks):
        x, y = blocks[:, 0], blocks[:, 1]
        inside = (x + size <= w) & (y + size <= h)
        if size > min_tu:
            split = ~inside | (rng.random(len(blocks)) < p_split)
        else:
            split = np.zeros(len(blocks), dtype=bool)
        keep = blocks[~split]
        if len(keep):
            out.append(np.column_stack([keep, np.full(len(keep), size)]))
        if size == min_tu:
            break
        half = size // 2
        kids = blocks[split]
        kids = np.concatenate([kids + [0, 0], kids + [half, 0], kids + [0, half],
                               kids + [half, half]])
        kids = kids[(kids[:, 0] < w) & (kids[:, 1] < h)]
        blocks, size = kids, half
    if not out:
        return np.zeros((0, 3), dtype=np.int32)
    return np.concatenate(out).astype(np.int32)


def ar1_arena_image(h: int, w: int, seed: int, rho: float) -> np.ndarray:
    """One image of an arena: AR(1) field from ``seed`` with ``rho``, sigma 40,
    mean 128, as uint8 (h x w)."""
    return _to_u8(ar1_field(h, w, rho, rng_for(seed)), 40.0, 128.0)


def ar1_arena(offsets, heights, widths, pitches, seeds, rhos, total: int, workers: int = 1):
    """Fill a flat uint8 arena with AR(1) images (sigma 40, mean 128) at the
    given pixel offsets, image i drawn from seed ``seeds[i]`` with ``rhos[i]``.
    Padding between rows and images is zero.  ``workers`` > 1 draws the
    images on that many threads (no process is forked)."""
    jobs = list(zip(map(int, offsets), map(int, heights), map(int, widths), map(int, pitches),
                    map(int, seeds), map(float, rhos)))
    arena = np.zeros(total, dtype=np.uint8)

    def one(job):
        off, h, w, pitch, seed, rho = job
        arena[off:off + pitch * h].reshape(h, pitch)[:, :w] = ar1_arena_image(h, w, seed, rho)

    # largest images first so that the threads stay balanced
    _run_threads(one, sorted(jobs, key=lambda j: -j[1] * j[2]), workers)
    return arena


def ragged_sizes(n: int, seed: int, median: float = 512.0, sigma: float = 0.75,
                 lo: int = 64, hi: int = 4096, mult: int = 8) -> np.ndarray:
    """``n`` (height, width) pairs, each side log-normal in [lo, hi], floored
    to a multiple of ``mult``."""
    rng = rng_for(seed)
    out = np.empty((n, 2), dtype=np.int64)
    for i in range(n):
        for j in range(2):
            while True:
                v = rng.lognormal(np.log(median), sigma)
                if lo <= v <= hi:
                    break
            out[i, j] = int(v) // mult * mult
    return out


def poisson_arrivals(n: int, rate_hz: float, seed: int) -> np.ndarray:
    """Arrival times (seconds, float64) of a Poisson process."""
    rng = rng_for(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def serving_requests(n: int, seed: int = 4000, rate_hz: float = 2000.0,
                     median: float = 1024.0, sigma: float = 0.5,
                     lo: int = 64, hi: int = 4096):
    """Request trace for the serving loop.

    Returns a list of dicts with keys ``t`` (arrival, s), ``h``, ``w``,
    ``transform`` (1 or 2), ``n`` (8/16/32), ``r`` (6..28) and ``seed``
    (content seed).  Sides are multiples of 32 so that every N fits.
    """
    rng = rng_for(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    reqs = []
    for i in range(n):
        hw = []
        for _ in range(2):
            while True:
                v = rng.lognormal(np.log(median), sigma)
                if lo <= v <= hi:
                    break
            hw.append(max(32, int(v) // 32 * 32))
        reqs.append(dict(t=float(t[i]), h=hw[0], w=hw[1],
                         transform=int(rng.integers(1, 3)),
                         n=int((8, 16, 32)[rng.integers(0, 3)]),
                         r=int(rng.integers(6, 29)),
                         seed=int(seed * 100000 + i)))
    return reqs
