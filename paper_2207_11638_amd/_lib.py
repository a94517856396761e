"""ctypes binding of libadct.so (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libadct.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "adct.h")

ADCT_T1, ADCT_T2 = 1, 2
ADCT_WHT, ADCT_SDCT, ADCT_HT, ADCT_DCT = 3, 4, 5, 6
ADCT_U8, ADCT_I16 = 0, 1
STATUS = {0: "ADCT_OK", -1: "ADCT_E_ARG", -2: "ADCT_E_SHAPE", -3: "ADCT_E_ALIGN",
          -4: "ADCT_E_HIP", -5: "ADCT_E_BUDGET"}

_i32, _i64, _vp = C.c_int, C.c_int64, C.c_void_p
_SIGNATURES = {
    "adct_version": ([], _i32),
    "adct_last_error": ([], C.c_char_p),
    "adct_get_matrix": ([_i32, _i32, _i32, _vp], _i32),
    "adct_zigzag": ([_i32, _vp], _i32),
    "adct_transform_measures": ([_i32, _i32, _vp, _vp], _i32),
    "adct_scale_vector": ([_i32, _i32, _vp], _i32),
    "adct_quant_tables": ([_i32, _i32, _i32, _vp, _vp], _i32),
    "adct_fwd2d": ([_i32, _i32, _vp, _i32, _i32, _i32, _i32, _i64, _i64, _vp, _vp], _i32),
    "adct_inv2d": ([_i32, _i32, _i32, _i32, _vp, _vp, _i32, _i32, _i32, _i32, _i64, _i64, _vp],
                   _i32),
    "adct_decompress": ([_i32, _i32, _i32, _i32, _vp, _vp, _i32, _i32, _i32, _i32, _i64, _i64,
                         _vp], _i32),
    "adct_compress": ([_i32, _i32, _i32, _i32, _vp, _i32, _i32, _i32, _i32, _i64, _i64, _vp, _vp,
                       _vp, _vp, _vp], _i32),
    "adct_compress_mfma": ([_i32, _i32, _vp, _i32, _i32, _i32, _i64, _i64, _vp, _vp, _vp, _vp,
                            _vp], _i32),
    "adct_psnr": ([_i32, _i64, _vp, _vp, _vp], _i32),
    "adct_stream_ceiling": ([_i32, _vp, _vp, _i64, _i32, _i32, _vp], _i32),
    "adct_ssim": ([_vp, _vp, _i32, _i32, _i32, _i64, _i64, _vp, _vp, _vp], _i32),
    "adct_ape": ([_i32, _vp, _vp, _vp, _vp], _i32),
    "adct_compress_quality": ([_i32, _i32, _i32, _i32, _vp, _i32, _i32, _i32, _i32, _i64, _i64,
                               _vp, _vp, _vp, _vp, _vp, _i32, _vp, _i64, _vp], _i32),
    "adct_compress_quality_workspace": ([_i32, _i32, _i32], _i64),
    "adct_compress_quality_noalloc": ([_i32, _i32, _i32, _i32, _vp, _i32, _i32, _i32, _i32, _i64,
                                       _i64, _vp, _vp, _vp, _vp, _vp, _i32, _vp], _i32),
    "adct_moments": ([_i32, _i32, _vp, _i32, _i32, _i32, _i32, _i64, _i64, _vp, _vp], _i32),
    "adct_coding_gain": ([_i32, _i32, _i32, _i32, _vp, _vp, _vp], _i32),
    "adct_coding_gain_ar1": ([_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp], _i32),
    "adct_batch_create": ([_vp, _i32, _vp, _i64, _i32, _vp, _vp, _vp], _i32),
    "adct_batch_destroy": ([_vp], _i32),
    "adct_batch_run": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp], _i32),
    "adct_batch_set_shape": ([_vp, _i32, _i32], _i32),
    "adct_batch_set_small_shape": ([_vp, _i32, _i32, _i32, _i32], _i32),
    "adct_batch_tune": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "adct_batch_info": ([_vp, _vp], _i32),
    "adct_server_create": ([_i64, _i32, _i32, _vp, _vp], _i32),
    "adct_server_destroy": ([_vp], _i32),
    "adct_server_submit": ([_vp, _vp], _i32),
    "adct_server_flush": ([_vp, _vp], _i32),
    "adct_server_poll": ([_vp, _i32, _vp, _i32, _vp], _i32),
    "adct_server_stats": ([_vp, _vp], _i32),
    "adct_server_clock_ms": ([_vp], C.c_double),
    "adct_server_run_trace": ([_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp], _i32),
}

ADCT_BASIS_ROWS, ADCT_BASIS_COLS = 0, 1


def moment_words(n: int) -> int:
    """uint64 words of one moment record (ADCT_MOMENT_WORDS)."""
    return 3 * n * n + 4


ADCT_RUN_BATCHED, ADCT_RUN_GRAPH, ADCT_RUN_PER_IMAGE, ADCT_RUN_UNIFIED = 0, 1, 2, 3

_lib = None


class AdctError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def header_functions() -> list:
    """Names of every function ``include/adct.h`` declares."""
    with open(HEADER) as f:
        text = f.read()
    return re.findall(r"ADCT_API\s+[\w\s\*]+?\b(adct_\w+)\s*\(", text)


def load() -> C.CDLL:
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "paper_2207_11638_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != 0:
        msg = load().adct_last_error()
        raise AdctError(status, msg.decode() if msg else "")
