"""ctypes mirror of ``include/huff.h``: structs, prototypes, library loading."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhuff.so")

ERRORS = {0: "HUFF_OK", -1: "HUFF_E_INVAL", -2: "HUFF_E_CAPACITY", -3: "HUFF_E_CORRUPT", -4: "HUFF_E_NOMEM",
          -5: "HUFF_E_AGAIN", -6: "HUFF_E_HIP", -7: "HUFF_E_CODELEN", -8: "HUFF_E_NOTFOUND", -9: "HUFF_E_MISMATCH"}
HUFF_OK, HUFF_E_INVAL, HUFF_E_CAPACITY, HUFF_E_CORRUPT, HUFF_E_NOMEM = 0, -1, -2, -3, -4
HUFF_E_AGAIN, HUFF_E_HIP, HUFF_E_CODELEN, HUFF_E_NOTFOUND, HUFF_E_MISMATCH = -5, -6, -7, -8, -9
#: kernel ids of huff_ctx_kernel_time
#: largest block of huff_bwt (HUFF_BWT_MAX_BLOCK)
HUFF_BWT_MAX_BLOCK = 16384
#: largest input of huff_compress_noalloc (HUFF_NOALLOC_MAX_N)
HUFF_NOALLOC_MAX_N = 256 << 20
HUFF_K_HIST, HUFF_K_CODEBOOK, HUFF_K_SCAN, HUFF_K_ENCODE, HUFF_K_DECODE = 0, 1, 2, 3, 4
KERNEL_IDS = {"hist": 0, "codebook": 1, "scan": 2, "encode": 3, "decode": 4}


class HuffError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {ERRORS.get(code, code)}")
        self.code = code


class HuffCodebook(ctypes.Structure):
    _fields_ = [("len", ctypes.c_uint8 * 256), ("code", ctypes.c_uint64 * 256), ("nsym", ctypes.c_uint32),
                ("max_len", ctypes.c_uint32)]


class HuffDcb(ctypes.Structure):
    _fields_ = [("nsym", ctypes.c_uint32), ("max_len", ctypes.c_uint32), ("lut_bits", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("total_bits", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("len", ctypes.c_uint8 * 256), ("sorted_sym", ctypes.c_uint8 * 256), ("code", ctypes.c_uint64 * 256),
                ("first_code", ctypes.c_uint64 * 64), ("first_index", ctypes.c_uint32 * 64),
                ("count", ctypes.c_uint32 * 64), ("enc", ctypes.c_uint32 * 256), ("lut", ctypes.c_uint16 * 1024)]


class HuffParams(ctypes.Structure):
    _fields_ = [("hist_blocks", ctypes.c_uint32), ("hist_depth", ctypes.c_uint32), ("dec_block", ctypes.c_uint32),
                ("enc_blocks_per_cu", ctypes.c_uint32)]


class HuffFile(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("n", ctypes.c_uint64), ("cb", ctypes.c_void_p), ("words", ctypes.c_void_p),
                ("cap_words", ctypes.c_uint64), ("chunk_off", ctypes.c_void_p), ("sub_lo", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("hist", ctypes.c_void_p), ("status", ctypes.c_void_p)]


HUFF_OP_COMPRESS, HUFF_OP_ENCODE, HUFF_OP_DECODE = 0, 1, 2


class HuffServerCfg(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_uint64), ("nslots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("chunk_size", ctypes.c_uint32), ("sub_size", ctypes.c_uint32)]


class HuffRequest(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("flags", ctypes.c_uint32), ("d_in", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("stream_handle", ctypes.c_uint64), ("d_expect", ctypes.c_void_p), ("expect_bits", ctypes.c_uint64)]


HUFF_REQ_DISCARD = 1


class HuffResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("handle", ctypes.c_uint64), ("in_bytes", ctypes.c_uint64),
                ("out_bytes", ctypes.c_uint64), ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class HuffStreamInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("total_bits", ctypes.c_uint64), ("cb", ctypes.c_void_p),
                ("words", ctypes.c_void_p), ("chunk_off", ctypes.c_void_p), ("sub_lo", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]

#: every symbol include/huff.h declares, with (restype, argtypes)
_vp, _u64, _u32, _i32, _int = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int
PROTOTYPES = {
    "huff_strerror": (ctypes.c_char_p, [_i32]),
    "huff_ctx_create": (_i32, [_int, _vp, _vp]),
    "huff_ctx_destroy": (None, [_vp]),
    "huff_ctx_set_params": (_i32, [_vp, _vp]),
    "huff_ctx_get_params": (_i32, [_vp, _vp]),
    "huff_ctx_status": (_i32, [_vp, _vp, _int]),
    "huff_ctx_set_timing": (_i32, [_vp, _int]),
    "huff_ctx_kernel_time": (_i32, [_vp, _int, _vp, _vp, _int]),
    "huff_histogram": (_i32, [_vp, _vp, _u64, _vp, _vp]),
    "huff_build_codebook": (_i32, [_vp, _vp]),
    "huff_encoded_bits": (_u64, [_vp, _vp]),
    "huff_build_codebook_device": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "huff_codebook_upload": (_i32, [_vp, _vp, _vp, _vp]),
    "huff_encode": (_i32, [_vp, _vp, _u64, _vp, _u32, _vp, _u64, _vp, _u32, _vp, _vp, _vp]),
    "huff_compress": (_i32, [_vp, _vp, _u64, _u32, _vp, _vp, _vp, _u64, _vp, _u32, _vp, _vp, _vp]),
    "huff_compress_noalloc": (_i32, [_vp, _vp, _u64, _u32, _vp, _vp, _vp, _u64, _vp, _u32, _vp, _vp, _vp]),
    "huff_decode": (_i32, [_vp, _vp, _u64, _vp, _u64, _u32, _vp, _u32, _vp, _vp, _vp, _vp]),
    "huff_copy": (_i32, [_vp, _vp, _vp, _u64, _vp]),
    "huff_bwt": (_i32, [_vp, _vp, _u64, _u32, _u32, _vp, _vp, _vp]),
    "huff_unbwt": (_i32, [_vp, _vp, _u64, _u32, _u32, _vp, _vp, _vp, _vp]),
    "huff_mtf": (_i32, [_vp, _vp, _u64, _u32, _vp, _vp]),
    "huff_unmtf": (_i32, [_vp, _vp, _u64, _u32, _vp, _vp]),
    "huff_abi_sizeof": (_u64, [_int]),
    "huff_batch_create": (_i32, [_vp, _vp, _u32, _u32, _u32, _vp]),
    "huff_batch_destroy": (None, [_vp]),
    "huff_batch_run": (_i32, [_vp, _int, _int, _vp]),
    "huff_compress_batch": (_i32, [_vp, _vp]),
    "huff_encode_batch": (_i32, [_vp, _vp]),
    "huff_decode_batch": (_i32, [_vp, _vp]),
    "huff_server_create": (_i32, [_vp, _vp, _vp]),
    "huff_server_submit": (_i32, [_vp, _vp, _vp]),
    "huff_server_poll": (_i32, [_vp, _u64, _vp]),
    "huff_server_wait": (_i32, [_vp, _u64, _vp]),
    "huff_server_stream": (_i32, [_vp, _u64, _vp]),
    "huff_server_release": (_i32, [_vp, _u64]),
    "huff_server_replay": (_i32, [_vp, _vp, _vp, _u32, _vp]),
    "huff_server_stats": (_i32, [_vp, _vp]),
    "huff_server_destroy": (None, [_vp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libhuff.so and binds every prototype.  Raises if it is missing:
    the codec has no other implementation to fall back to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    l = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(l, name)
        fn.restype = res
        fn.argtypes = args
    for i, cls in enumerate((HuffDcb, HuffCodebook, HuffParams, HuffFile, HuffServerCfg, HuffRequest, HuffResult,
                             HuffStreamInfo)):
        if l.huff_abi_sizeof(i) != ctypes.sizeof(cls):
            raise ImportError(f"ABI mismatch for {cls.__name__}: C {l.huff_abi_sizeof(i)} vs ctypes {ctypes.sizeof(cls)}")
    _lib = l
    return l


def lib():
    return load()
