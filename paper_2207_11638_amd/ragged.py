"""Packing of ragged image sets into the pixel arenas a BatchPlan addresses."""
from __future__ import annotations

import numpy as np

from . import IMAGE_DESC, TU_DESC


def pack_images(images, transforms, rs, qsteps=None, align_bytes: int = 256):
    """Concatenate 2D arrays (all uint8 or all int16) into one flat arena.

    Each image starts at an ``align_bytes`` boundary and its rows are padded
    to a 16-byte multiple.  Returns ``(arena, descs)``: the 1D numpy arena
    and an IMAGE_DESC array with the same offsets for source and
    reconstruction (use an arena of the same size for the latter).
    """
    n = len(images)
    if n == 0:
        return np.zeros(0, dtype=np.uint8), np.zeros(0, dtype=IMAGE_DESC)
    dt = images[0].dtype
    esize = dt.itemsize
    qsteps = [0] * n if qsteps is None else qsteps
    descs = np.zeros(n, dtype=IMAGE_DESC)
    off = 0
    for i, im in enumerate(images):
        h, w = im.shape
        pitch = -(-w * esize // 16) * 16 // esize
        off = -(-off * esize // align_bytes) * align_bytes // esize
        descs[i] = (off, off, h, w, pitch, int(transforms[i]), int(rs[i]), int(qsteps[i]))
        off += pitch * h
    arena = np.zeros(off, dtype=dt)
    for i, im in enumerate(images):
        o, p = int(descs[i]["src_offset"]), int(descs[i]["pitch"])
        h, w = im.shape
        arena[o:o + p * h].reshape(h, p)[:, :w] = im
    return arena, descs


def unpack_image(arena: np.ndarray, desc) -> np.ndarray:
    o, p, h, w = int(desc["dst_offset"]), int(desc["pitch"]), int(desc["height"]), int(desc["width"])
    return arena[o:o + p * h].reshape(h, p)[:, :w]


def tu_table(per_image_tus) -> np.ndarray:
    """Stack per-image (x, y, n) arrays into one TU_DESC array."""
    rows = []
    for i, t in enumerate(per_image_tus):
        t = np.asarray(t, dtype=np.int32).reshape(-1, 3)
        out = np.zeros(len(t), dtype=TU_DESC)
        out["image"] = i
        out["x"], out["y"], out["n"] = t[:, 0], t[:, 1], t[:, 2]
        rows.append(out)
    return np.concatenate(rows) if rows else np.zeros(0, dtype=TU_DESC)
