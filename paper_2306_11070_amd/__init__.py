"""Python binding of the MI355X Huffman codec (``libhuff.so``, C ABI in
``include/huff.h``).

Argument marshalling only: every step of the codec runs in the HIP kernels
of the library.  PyTorch supplies device memory and streams.  If the library
is not built, or a call fails, this module raises; it never falls back to a
CPU implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from ._abi import (HuffCodebook, HuffDcb, HuffParams, ERRORS, HuffError, lib, load)

__all__ = ["Codec", "HuffError", "build_codebook", "encoded_bits", "dcb_to_host", "load", "DCB_BYTES"]

DCB_BYTES = ctypes.sizeof(HuffDcb)


def _torch():
    import torch
    return torch


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _check(rc: int, what: str):
    if rc != 0:
        raise HuffError(rc, what)


def build_codebook(hist) -> HuffCodebook:
    """Host codebook (tie-ruled Huffman lengths + canonical codes)."""
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    assert h.size == 256
    cb = HuffCodebook()
    _check(lib().huff_build_codebook(h.ctypes.data, ctypes.byref(cb)), "huff_build_codebook")
    return cb


def encoded_bits(hist, cb: HuffCodebook) -> int:
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    return int(lib().huff_encoded_bits(h.ctypes.data, ctypes.byref(cb)))


def dcb_to_host(dcb) -> HuffDcb:
    """Copies a device codebook tensor back and parses it (synchronises)."""
    raw = dcb.detach().cpu().numpy().tobytes()
    return HuffDcb.from_buffer_copy(raw[:DCB_BYTES])


class Codec:
    """One context (device workspaces) of the library on one HIP device.

    Calls queue work on ``stream`` (default: torch's current stream) and
    return without waiting.  A context's calls must be ordered on one stream
    at a time.
    """

    def __init__(self, device: int = 0, params: dict | None = None):
        torch = _torch()
        self.device = torch.device("cuda", device)
        p = HuffParams(**(params or {}))
        ctx = ctypes.c_void_p()
        _check(lib().huff_ctx_create(device, ctypes.byref(p), ctypes.byref(ctx)), "huff_ctx_create")
        self._ctx = ctx

    def close(self):
        if self._ctx:
            lib().huff_ctx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------
    def _stream(self, stream):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(int(s.cuda_stream))

    def _u8(self, x):
        torch = _torch()
        assert x.dtype == torch.uint8 and x.is_cuda and x.is_contiguous(), "expected a contiguous cuda uint8 tensor"
        return x

    @property
    def params(self) -> dict:
        p = HuffParams()
        _check(lib().huff_ctx_get_params(self._ctx, ctypes.byref(p)), "huff_ctx_get_params")
        return {k: getattr(p, k) for k, _ in HuffParams._fields_}

    def set_params(self, **kw):
        p = HuffParams(**kw)
        _check(lib().huff_ctx_set_params(self._ctx, ctypes.byref(p)), "huff_ctx_set_params")

    def status(self, reset: bool = True) -> int:
        """Waits for the device and returns (and clears) the context status word."""
        out = ctypes.c_int32()
        _check(lib().huff_ctx_status(self._ctx, ctypes.byref(out), int(reset)), "huff_ctx_status")
        return out.value

    def new_status(self):
        torch = _torch()
        return torch.zeros(1, dtype=torch.int32, device=self.device)

    # -- the path ------------------------------------------------------------
    def histogram(self, x, out=None, stream=None):
        torch = _torch()
        x = self._u8(x)
        if out is None:
            out = torch.empty(256, dtype=torch.int64, device=self.device)
        _check(lib().huff_histogram(self._ctx, _ptr(x), x.numel(), _ptr(out), self._stream(stream)), "huff_histogram")
        return out

    def build_codebook_device(self, hist, out=None, status=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(DCB_BYTES, dtype=torch.uint8, device=self.device)
        _check(lib().huff_build_codebook_device(self._ctx, _ptr(hist), _ptr(out), _ptr(status), self._stream(stream)),
               "huff_build_codebook_device")
        return out

    def codebook_upload(self, cb: HuffCodebook, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(DCB_BYTES, dtype=torch.uint8, device=self.device)
        _check(lib().huff_codebook_upload(self._ctx, ctypes.byref(cb), _ptr(out), self._stream(stream)),
               "huff_codebook_upload")
        return out

    def encode(self, x, dcb, chunk_size: int, sub_size: int = 0, words=None, chunk_off=None, sub_lo=None,
               status=None, stream=None):
        """Returns (words int32 view of u32, chunk_off int64 view of u64, sub_lo or None)."""
        torch = _torch()
        x = self._u8(x)
        n = x.numel()
        if words is None:
            words = torch.empty((n + 3) // 4 + 4, dtype=torch.int32, device=self.device)
        nch = (n + chunk_size - 1) // chunk_size
        if chunk_off is None:
            chunk_off = torch.empty(nch + 1, dtype=torch.int64, device=self.device)
        if sub_size and sub_lo is None:
            sub_lo = torch.empty((n + sub_size - 1) // sub_size + 1, dtype=torch.int32, device=self.device)
        _check(lib().huff_encode(self._ctx, _ptr(x), n, _ptr(dcb), chunk_size, _ptr(words), words.numel(),
                                 _ptr(chunk_off), sub_size, _ptr(sub_lo) if sub_size else None, _ptr(status),
                                 self._stream(stream)), "huff_encode")
        return words, chunk_off, (sub_lo if sub_size else None)

    def decode(self, words, nwords: int, chunk_off, n: int, chunk_size: int, dcb, sub_lo=None, sub_size: int = 0,
               out=None, status=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().huff_decode(self._ctx, _ptr(words), nwords, _ptr(chunk_off), n, chunk_size,
                                 _ptr(sub_lo) if sub_size else None, sub_size, _ptr(dcb), _ptr(out), _ptr(status),
                                 self._stream(stream)), "huff_decode")
        return out

    def copy(self, src, dst, nbytes: int | None = None, stream=None):
        nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
        _check(lib().huff_copy(self._ctx, _ptr(src), _ptr(dst), nbytes, self._stream(stream)), "huff_copy")

    # -- whole path conveniences (still only library calls) -------------------
    def compress(self, x, chunk_size: int, sub_size: int = 0, status=None, stream=None, out: dict | None = None) -> dict:
        """huff_compress: histogram, device codebook and encode in one call.
        `out` may hold preallocated hist/dcb/words/chunk_off/sub_lo tensors."""
        torch = _torch()
        x = self._u8(x)
        n = x.numel()
        o = dict(out or {})
        hist = o.get("hist")
        if hist is None:
            hist = torch.empty(256, dtype=torch.int64, device=self.device)
        dcb = o.get("dcb")
        if dcb is None:
            dcb = torch.empty(DCB_BYTES, dtype=torch.uint8, device=self.device)
        words = o.get("words")
        if words is None:
            words = torch.empty((n + 3) // 4 + 4, dtype=torch.int32, device=self.device)
        off = o.get("chunk_off")
        if off is None:
            off = torch.empty((n + chunk_size - 1) // chunk_size + 1, dtype=torch.int64, device=self.device)
        sub = o.get("sub_lo")
        if sub_size and sub is None:
            sub = torch.empty((n + sub_size - 1) // sub_size + 1, dtype=torch.int32, device=self.device)
        _check(lib().huff_compress(self._ctx, _ptr(x), n, chunk_size, _ptr(dcb), _ptr(hist), _ptr(words), words.numel(),
                                   _ptr(off), sub_size, _ptr(sub) if sub_size else None, _ptr(status),
                                   self._stream(stream)), "huff_compress")
        return dict(hist=hist, dcb=dcb, words=words, chunk_off=off, sub_lo=sub if sub_size else None, n=n,
                    chunk_size=chunk_size, sub_size=sub_size)

    def decompress(self, c: dict, out=None, status=None, stream=None):
        return self.decode(c["words"], c["words"].numel(), c["chunk_off"], c["n"], c["chunk_size"], c["dcb"],
                           c.get("sub_lo"), c.get("sub_size", 0), out=out, status=status, stream=stream)
