"""Block-wise Chen-based approximate DCT on MI355X (gfx950).

Python front end of ``libadct.so``: it checks tensor placement and shapes,
allocates outputs with PyTorch and passes raw device pointers and the current
HIP stream to the C ABI declared in ``include/adct.h``.  Every step of the
transform runs in the library's HIP kernels; there is no CPU path.

Transforms (section 3 and section 6.1 of the paper):
  T1 = the sign-based approximation T~_N (eq. 4 for N = 8),
  T2 = the round-based approximation T^_N (eq. 5 for N = 8),
  N in {8, 16, 32}; N = 16, 32 use the Chen-JAM recursion.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (ADCT_DCT, ADCT_HT, ADCT_I16, ADCT_SDCT, ADCT_T1, ADCT_T2, ADCT_U8, ADCT_WHT,
                   AdctError)

__all__ = ["ADCT_T1", "ADCT_T2", "ADCT_WHT", "ADCT_SDCT", "ADCT_HT", "ADCT_DCT", "AdctError", "get_matrix", "zigzag", "scale_vector",
           "quant_tables", "transform_measures", "fwd2d", "inv2d", "compress", "decompress", "library_path",
           "psnr", "moments", "coding_gain", "coding_gain_ar1", "compress_quality", "ssim", "ape",
           "BatchPlan", "IMAGE_DESC", "TU_DESC"]

library_path = _lib.LIB_PATH


# ----------------------------------------------------------------- host queries
def get_matrix(transform: int, n: int, inverse: bool = False) -> np.ndarray:
    """T_N (or U_N = N T_N^-1) as computed by the library's butterflies."""
    out = np.zeros((n, n), dtype=np.int32)
    _lib.check(_lib.load().adct_get_matrix(transform, n, int(inverse), out.ctypes.data))
    return out


def zigzag(n: int) -> np.ndarray:
    out = np.zeros(n * n, dtype=np.int32)
    _lib.check(_lib.load().adct_zigzag(n, out.ctypes.data))
    return out


def scale_vector(transform: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    _lib.check(_lib.load().adct_scale_vector(transform, n, out.ctypes.data))
    return out


def transform_measures(transform: int, n: int):
    """(total error energy against the DCT, deviation from diagonality of
    T T^T) of the library's transform (section 4.1, Table 1)."""
    eps = C.c_double()
    delta = C.c_double()
    _lib.check(_lib.load().adct_transform_measures(transform, n, C.byref(eps), C.byref(delta)))
    return eps.value, delta.value


def quant_tables(transform: int, n: int, qstep: int):
    mq = np.zeros((n, n), dtype=np.int32)
    dq = np.zeros((n, n), dtype=np.int32)
    _lib.check(_lib.load().adct_quant_tables(transform, n, qstep, mq.ctypes.data,
                                             dq.ctypes.data))
    return mq, dq


# ----------------------------------------------------------------- device calls
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.uint8:
        return ADCT_U8
    if t.dtype == torch.int16:
        return ADCT_I16
    raise TypeError(f"pixels must be uint8 or int16, got {t.dtype}")


def _image_geometry(x):
    """(batch, height, width, pitch, image_stride) of a [B,H,W] or [H,W] tensor."""
    if x.dim() == 2:
        x = x.unsqueeze(0)
    if x.dim() != 3:
        raise ValueError("images must be [H, W] or [B, H, W]")
    if x.stride(2) != 1:
        raise ValueError("image rows must be contiguous")
    b, h, w = x.shape
    return b, h, w, x.stride(1), (x.stride(0) if b > 1 else x.stride(1) * h)


def _require_device(*tensors):
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise ValueError("libadct runs on the GPU only: pass device tensors")


def _stream_handle(device) -> C.c_void_p:
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def fwd2d(x, transform: int, n: int, out=None):
    """All coefficients of every tile: int32 [B, H/n, W/n, n, n]."""
    torch = _torch()
    _require_device(x, out)
    b, h, w, pitch, istride = _image_geometry(x)
    if out is None:
        out = torch.empty((b, h // n, w // n, n, n), dtype=torch.int32, device=x.device)
    _lib.check(_lib.load().adct_fwd2d(transform, n, _ptr(x), _dtype_code(x), b, h, w, pitch,
                                      istride, _ptr(out), _stream_handle(x.device)))
    return out


def inv2d(coef, transform: int, n: int, r: int, qstep: int = 0, dtype=None, out=None):
    """Reconstruct images from natural-order coefficients [B, H/n, W/n, n, n]."""
    torch = _torch()
    _require_device(coef, out)
    if coef.dtype != torch.int32 or not coef.is_contiguous() or coef.dim() != 5:
        raise ValueError("coefficients must be a contiguous int32 [B, H/n, W/n, n, n] tensor")
    b, th, tw = coef.shape[:3]
    if out is None:
        out = torch.empty((b, th * n, tw * n), dtype=dtype or torch.uint8, device=coef.device)
    ob, h, w, pitch, istride = _image_geometry(out)
    _lib.check(_lib.load().adct_inv2d(transform, n, r, qstep, _ptr(coef), _ptr(out),
                                      _dtype_code(out), ob, h, w, pitch, istride,
                                      _stream_handle(coef.device)))
    return out


def compress(x, transform: int, n: int, r: int, qstep: int = 0, *, kept=True, scaled=True,
             recon=True, sse=True, engine: str = "butterfly"):
    """The fused pipeline.  Each of kept/scaled/recon/sse may be True (allocate),
    False (skip) or a preallocated tensor.  Returns a dict of the produced
    tensors: kept int32 [B, H/n, W/n, r], scaled float32 [B, H/n, W/n, r],
    recon like x, sse uint64 [B] (accumulated into when passed in).
    engine="mfma" runs the int8 matrix-core form (n = 8, uint8, qstep = 0).
    The exact DCT (ADCT_DCT) has no integer coefficients: kept defaults to
    False and scaled holds its orthonormal coefficients."""
    if engine not in ("butterfly", "mfma"):
        raise ValueError(f"unknown engine {engine!r}")
    torch = _torch()
    _require_device(x)
    b, h, w, pitch, istride = _image_geometry(x)
    dev = x.device
    tiles = (b, h // n, w // n)

    def pick(v, make):
        if v is True:
            return make()
        if v is False or v is None:
            return None
        _require_device(v)
        return v

    if transform == ADCT_DCT and kept is True:
        kept = False
    kept_t = pick(kept, lambda: torch.empty(tiles + (r,), dtype=torch.int32, device=dev))
    scaled_t = pick(scaled, lambda: torch.empty(tiles + (r,), dtype=torch.float32, device=dev))
    recon_t = pick(recon, lambda: torch.empty_strided(x.size(), x.stride(), dtype=x.dtype,
                                                        device=dev))
    sse_t = pick(sse, lambda: torch.zeros(b, dtype=torch.uint64, device=dev))
    if recon_t is not None:
        rb, rh, rw, rp, rs = _image_geometry(recon_t)
        if (rb, rh, rw, rp, rs) != (b, h, w, pitch, istride):
            raise ValueError("recon must have the geometry of x")
    if engine == "mfma":
        if n != 8 or qstep != 0 or x.dtype != torch.uint8:
            raise ValueError("the mfma engine takes n = 8, uint8 images and qstep = 0")
        _lib.check(_lib.load().adct_compress_mfma(transform, r, _ptr(x), b, h, w, pitch, istride,
                                                  _ptr(kept_t), _ptr(scaled_t), _ptr(recon_t),
                                                  _ptr(sse_t), _stream_handle(dev)))
    else:
        _lib.check(_lib.load().adct_compress(transform, n, r, qstep, _ptr(x), _dtype_code(x), b,
                                             h, w, pitch, istride, _ptr(kept_t), _ptr(scaled_t),
                                             _ptr(recon_t), _ptr(sse_t), _stream_handle(dev)))
    return {"kept": kept_t, "scaled": scaled_t, "recon": recon_t, "sse": sse_t}


def decompress(kept, transform: int, n: int, r: int, qstep: int = 0, dtype=None, out=None):
    """Reconstruct from zig-zag-ordered retained coefficients [B, H/n, W/n, r]."""
    torch = _torch()
    _require_device(kept, out)
    if kept.dtype != torch.int32 or not kept.is_contiguous() or kept.dim() != 4:
        raise ValueError("kept must be a contiguous int32 [B, H/n, W/n, r] tensor")
    b, th, tw, rr = kept.shape
    if rr != r:
        raise ValueError("kept.shape[-1] must equal r")
    if out is None:
        out = torch.empty((b, th * n, tw * n), dtype=dtype or torch.uint8, device=kept.device)
    ob, h, w, pitch, istride = _image_geometry(out)
    _lib.check(_lib.load().adct_decompress(transform, n, r, qstep, _ptr(kept), _ptr(out),
                                           _dtype_code(out), ob, h, w, pitch, istride,
                                           _stream_handle(kept.device)))
    return out


# ----------------------------------------------------------------- quality measures
_BASES = {"rows": _lib.ADCT_BASIS_ROWS, "cols": _lib.ADCT_BASIS_COLS}


def _basis_code(basis: str) -> int:
    if basis not in _BASES:
        raise ValueError(f"basis must be 'rows' or 'cols', got {basis!r}")
    return _BASES[basis]


def psnr(sse, pixels: int, out=None):
    """float32 PSNR per image from uint64 error energies [B] (images of
    ``pixels`` pixels each); +inf where the error energy is zero."""
    torch = _torch()
    _require_device(sse, out)
    if sse.dtype != torch.uint64 or not sse.is_contiguous() or sse.dim() != 1:
        raise ValueError("sse must be a contiguous uint64 [B] tensor")
    if out is None:
        out = torch.empty(sse.numel(), dtype=torch.float32, device=sse.device)
    _lib.check(_lib.load().adct_psnr(sse.numel(), int(pixels), _ptr(sse), _ptr(out),
                                     _stream_handle(sse.device)))
    return out


def ssim(x, y):
    """float32 mean SSIM (11 x 11 Gaussian windows) of every image pair of two
    uint8 tensors of one geometry ([B, H, W] or [H, W])."""
    torch = _torch()
    _require_device(x, y)
    if x.dtype != torch.uint8 or y.dtype != torch.uint8:
        raise TypeError("SSIM takes uint8 images")
    b, h, w, pitch, istride = _image_geometry(x)
    if _image_geometry(y) != (b, h, w, pitch, istride):
        raise ValueError("x and y must have the same geometry")
    work = torch.empty(b, dtype=torch.float64, device=x.device)
    out = torch.empty(b, dtype=torch.float32, device=x.device)
    _lib.check(_lib.load().adct_ssim(_ptr(x), _ptr(y), b, h, w, pitch, istride, _ptr(work),
                                     _ptr(out), _stream_handle(x.device)))
    return out


def ape(value, reference):
    """float32 absolute percentage error of ``value`` against ``reference``."""
    torch = _torch()
    _require_device(value, reference)
    for t in (value, reference):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("APE takes contiguous float32 tensors")
    if value.numel() != reference.numel():
        raise ValueError("value and reference differ in size")
    out = torch.empty_like(value)
    _lib.check(_lib.load().adct_ape(value.numel(), _ptr(value), _ptr(reference), _ptr(out),
                                    _stream_handle(value.device)))
    return out


def moments(x, transform: int, n: int, out=None):
    """Coefficient and pixel moments of every image: uint64 [B, 3 n^2 + 4]
    (layout of adct_moments), accumulated into ``out`` when it is given."""
    torch = _torch()
    _require_device(x, out)
    b, h, w, pitch, istride = _image_geometry(x)
    if out is None:
        out = torch.zeros((b, _lib.moment_words(n)), dtype=torch.uint64, device=x.device)
    elif (out.dtype != torch.uint64 or not out.is_contiguous() or
          tuple(out.shape) != (b, _lib.moment_words(n))):
        raise ValueError("out must be a contiguous uint64 [B, 3 n^2 + 4] tensor")
    _lib.check(_lib.load().adct_moments(transform, n, _ptr(x), _dtype_code(x), b, h, w, pitch,
                                        istride, _ptr(out), _stream_handle(x.device)))
    return out


def coding_gain(mom, transform: int, n: int, basis: str = "cols", out=None):
    """Measured 2D coding gain (dB, float32) of every moment record [B, 3 n^2 + 4]."""
    torch = _torch()
    _require_device(mom, out)
    if (mom.dtype != torch.uint64 or not mom.is_contiguous() or mom.dim() != 2 or
            mom.shape[1] != _lib.moment_words(n)):
        raise ValueError("moments must be a contiguous uint64 [B, 3 n^2 + 4] tensor")
    if out is None:
        out = torch.empty(mom.shape[0], dtype=torch.float32, device=mom.device)
    _lib.check(_lib.load().adct_coding_gain(transform, n, _basis_code(basis), mom.shape[0],
                                            _ptr(mom), _ptr(out), _stream_handle(mom.device)))
    return out


def compress_quality(x, transform: int, n: int, r: int, qstep: int = 0, *, kept=True,
                     scaled=True, recon=True, coding_gain=True, basis: str = "cols"):
    """The fused pipeline plus the float32 PSNR and (optionally) the measured
    coding gain of every image, in one library call with a workspace the
    binding allocates.  Returns a dict: kept, scaled, recon (or None), psnr
    float32 [B], coding_gain float32 [B] (or None)."""
    torch = _torch()
    _require_device(x)
    b, h, w, pitch, istride = _image_geometry(x)
    dev = x.device
    tiles = (b, h // n, w // n)
    if transform == ADCT_DCT:   # no integer coefficients, no moments
        kept = coding_gain = False
    kept_t = torch.empty(tiles + (r,), dtype=torch.int32, device=dev) if kept else None
    scaled_t = torch.empty(tiles + (r,), dtype=torch.float32, device=dev) if scaled else None
    recon_t = (torch.empty_strided(x.size(), x.stride(), dtype=x.dtype, device=dev)
               if recon else None)
    psnr_t = torch.empty(b, dtype=torch.float32, device=dev)
    cg_t = torch.empty(b, dtype=torch.float32, device=dev) if coding_gain else None
    lib = _lib.load()
    nbytes = lib.adct_compress_quality_workspace(n, b, int(bool(coding_gain)))
    if nbytes < 0:
        _lib.check(int(nbytes))
    work = torch.empty(max(1, nbytes // 8), dtype=torch.uint64, device=dev)
    _lib.check(lib.adct_compress_quality(transform, n, r, qstep, _ptr(x), _dtype_code(x), b, h, w,
                                         pitch, istride, _ptr(kept_t), _ptr(scaled_t),
                                         _ptr(recon_t), _ptr(psnr_t), _ptr(cg_t),
                                         _basis_code(basis), _ptr(work), nbytes,
                                         _stream_handle(dev)))
    return {"kept": kept_t, "scaled": scaled_t, "recon": recon_t, "psnr": psnr_t,
            "coding_gain": cg_t}


def coding_gain_ar1(rho, transform: int, n: int, basis: str = "cols"):
    """Coding gain (dB, float32) of C = S' T under the AR(1) model for every
    correlation value in the float32 device tensor ``rho``; returns
    (gain, KLT gain)."""
    torch = _torch()
    _require_device(rho)
    if rho.dtype != torch.float32 or not rho.is_contiguous() or rho.dim() != 1:
        raise ValueError("rho must be a contiguous float32 vector")
    cg = torch.empty_like(rho)
    klt = torch.empty_like(rho)
    _lib.check(_lib.load().adct_coding_gain_ar1(transform, n, _basis_code(basis), rho.numel(),
                                                _ptr(rho), _ptr(cg), _ptr(klt),
                                                _stream_handle(rho.device)))
    return cg, klt


# ----------------------------------------------------------------- ragged batches
# numpy mirrors of adct_image_desc_t and adct_tu_desc_t
IMAGE_DESC = np.dtype([("src_offset", np.int64), ("dst_offset", np.int64), ("height", np.int32),
                       ("width", np.int32), ("pitch", np.int32), ("transform", np.int32),
                       ("r", np.int32), ("qstep", np.int32)])
TU_DESC = np.dtype([("image", np.int32), ("x", np.int32), ("y", np.int32), ("n", np.int32)])

_RUN_MODES = {"batched": _lib.ADCT_RUN_BATCHED, "graph": _lib.ADCT_RUN_GRAPH,
              "per_image": _lib.ADCT_RUN_PER_IMAGE, "unified": _lib.ADCT_RUN_UNIFIED}


class BatchPlan:
    """A plan for many images, each split into 8/16/32 transform units.

    images: structured array of IMAGE_DESC (offsets in pixels into the source
    and reconstruction arenas); tus: structured array of TU_DESC; dtype:
    torch.uint8 or torch.int16.  After construction ``kept_words`` is the
    length of the retained-coefficient arena and ``tu_kept_offset[t]`` the
    first word of TU t in it."""

    def __init__(self, images, tus, dtype):
        torch = _torch()
        self.images = np.ascontiguousarray(images, dtype=IMAGE_DESC)
        self.tus = np.ascontiguousarray(tus, dtype=TU_DESC)
        code = ADCT_U8 if dtype == torch.uint8 else ADCT_I16
        self.dtype = dtype
        self.tu_kept_offset = np.zeros(len(self.tus), dtype=np.int64)
        words = C.c_int64(0)
        handle = C.c_void_p()
        _lib.check(_lib.load().adct_batch_create(
            self.images.ctypes.data, len(self.images), self.tus.ctypes.data, len(self.tus), code,
            self.tu_kept_offset.ctypes.data, C.byref(words), C.byref(handle)))
        self._h = handle
        self.kept_words = int(words.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().adct_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        out = np.zeros(14, dtype=np.int64)
        _lib.check(_lib.load().adct_batch_info(self._h, out.ctypes.data))
        keys = ("images", "tus", "items", "items8", "items16", "items32", "buckets", "cus",
                "unified_items", "small_bound", "small_groups8", "small_groups16",
                "persistent", "wgs_per_cu")
        return dict(zip(keys, out.tolist()))

    def set_shape(self, bs8: int, bs_jam: int):
        _lib.check(_lib.load().adct_batch_set_shape(self._h, bs8, bs_jam))

    def set_small_shape(self, groups8: int, groups16: int, persistent: bool = False,
                        wgs_per_cu: int = 8):
        """Shape of the row-per-thread unified launch (see adct.h)."""
        _lib.check(_lib.load().adct_batch_set_small_shape(self._h, groups8, groups16,
                                                          int(persistent), wgs_per_cu))

    def tune(self, src, dst=None, kept=None, scaled=None, sse=None):
        _require_device(src, dst, kept, scaled, sse)
        chosen = np.zeros(max(1, self.info()["buckets"]), dtype=np.int32)
        _lib.check(_lib.load().adct_batch_tune(self._h, _ptr(src), _ptr(dst), _ptr(kept),
                                               _ptr(scaled), _ptr(sse),
                                               _stream_handle(src.device), chosen.ctypes.data))
        return chosen

    def run(self, src, dst=None, kept=None, scaled=None, sse=None, psnr=None, mode="batched"):
        """Enqueue one pass over every TU on the current stream.  Buffers are
        device tensors (or None): src/dst pixel arenas, kept int32 / scaled
        float32 of kept_words words, sse uint64 / psnr float32 per image."""
        _require_device(src, dst, kept, scaled, sse, psnr)
        _lib.check(_lib.load().adct_batch_run(self._h, _ptr(src), _ptr(dst), _ptr(kept),
                                              _ptr(scaled), _ptr(sse), _ptr(psnr),
                                              _RUN_MODES[mode], _stream_handle(src.device)))


# ----------------------------------------------------------------- serving
# numpy mirrors of adct_request_t and adct_completion_t
REQUEST = np.dtype([("d_src", np.uint64), ("h_kept", np.uint64), ("h_scaled", np.uint64),
                    ("h_recon", np.uint64),
                    ("pitch", np.int64), ("tag", np.int64), ("transform", np.int32),
                    ("n", np.int32), ("r", np.int32), ("qstep", np.int32), ("dtype", np.int32),
                    ("height", np.int32), ("width", np.int32), ("want_scaled", np.int32)])
COMPLETION = np.dtype([("tag", np.int64), ("batch", np.int64), ("sse", np.uint64),
                       ("done_ms", np.float64), ("launch_ms", np.float64), ("d_kept", np.uint64),
                       ("d_scaled", np.uint64),
                       ("d_recon", np.uint64)])


def request(x, transform: int, n: int, r: int, qstep: int = 0, tag: int = 0,
            want_scaled: bool = False, h_kept=None, h_scaled=None, h_recon=None):
    """One REQUEST record for the 2D image tensor x (uint8 or int16 on the
    GPU, rows contiguous).  h_kept / h_scaled / h_recon: optional host
    tensors (pinned for an asynchronous copy) that receive the kept
    coefficients ([H/n * W/n * r] int32), the scaled coefficients (float32,
    needs want_scaled) and the reconstruction (x's rows, x's pitch)."""
    if x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("x must be a 2D tensor with contiguous rows")
    rec = np.zeros((), dtype=REQUEST)
    rec["d_src"] = x.data_ptr()
    rec["h_kept"] = 0 if h_kept is None else h_kept.data_ptr()
    rec["h_scaled"] = 0 if h_scaled is None else h_scaled.data_ptr()
    rec["h_recon"] = 0 if h_recon is None else h_recon.data_ptr()
    rec["pitch"] = x.stride(0)
    rec["tag"] = tag
    rec["transform"], rec["n"], rec["r"], rec["qstep"] = transform, n, r, qstep
    rec["dtype"] = _dtype_code(x)
    rec["height"], rec["width"] = x.shape
    rec["want_scaled"] = int(bool(want_scaled))
    return rec


class Server:
    """Continuous-batching compress server on one GPU stream (see the
    adct_server_* calls).  budget: HBM bytes charged by the requests in
    flight (inputs + outputs); max_inflight batch slots; max_batch requests
    per batch."""

    def __init__(self, budget: int, max_inflight: int = 2, max_batch: int = 1024, stream=None):
        handle = C.c_void_p()
        self.max_batch = max_batch
        _lib.check(_lib.load().adct_server_create(int(budget), max_inflight, max_batch,
                                                  stream, C.byref(handle)))
        self._h = handle
        self._out = np.zeros(max_batch, dtype=COMPLETION)

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().adct_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, rec) -> bool:
        """Queue one request; False when the budget cannot take it now."""
        rec = np.ascontiguousarray(rec, dtype=REQUEST)
        st = _lib.load().adct_server_submit(self._h, rec.ctypes.data)
        if st == -5:
            return False
        _lib.check(st)
        return True

    def flush(self) -> int:
        launched = C.c_int(0)
        _lib.check(_lib.load().adct_server_flush(self._h, C.byref(launched)))
        return launched.value

    def poll(self, wait: bool = False):
        """Completed requests (structured COMPLETION array), oldest first."""
        n = C.c_int(0)
        _lib.check(_lib.load().adct_server_poll(self._h, int(wait), self._out.ctypes.data,
                                                len(self._out), C.byref(n)))
        return self._out[: n.value].copy()

    def stats(self) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _lib.check(_lib.load().adct_server_stats(self._h, out.ctypes.data))
        keys = ("submitted", "completed", "batches", "queued", "in_flight", "charged",
                "max_batch", "refused")
        return dict(zip(keys, out.tolist()))

    def clock_ms(self) -> float:
        return float(_lib.load().adct_server_clock_ms(self._h))

    def run_trace(self, requests, arrival_ms, launch_times: bool = False):
        """Replay an arrival trace in real time (native loop); returns
        (latency_ms, batch_of, sse) arrays, and launch_ms (host time of each
        request's launch after the start) as a fourth when launch_times."""
        reqs = np.ascontiguousarray(requests, dtype=REQUEST)
        arr = np.ascontiguousarray(arrival_ms, dtype=np.float64)
        lat = np.zeros(len(reqs), dtype=np.float64)
        bat = np.zeros(len(reqs), dtype=np.int64)
        sse = np.zeros(len(reqs), dtype=np.uint64)
        launch = np.zeros(len(reqs), dtype=np.float64)
        _lib.check(_lib.load().adct_server_run_trace(self._h, reqs.ctypes.data, arr.ctypes.data,
                                                     len(reqs), lat.ctypes.data,
                                                     bat.ctypes.data, sse.ctypes.data,
                                                     launch.ctypes.data))
        return (lat, bat, sse, launch) if launch_times else (lat, bat, sse)
