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

from . import _abi
from ._abi import (HuffCodebook, HuffDcb, HuffFile, HuffParams, HuffRequest, HuffResult, HuffServerCfg,
                   HuffStreamInfo, ERRORS, HuffError, lib, load, HUFF_OP_COMPRESS, HUFF_OP_ENCODE, HUFF_OP_DECODE,
                   HUFF_E_AGAIN)

__all__ = ["Codec", "Batch", "Segments", "Server", "batch_buffers", "HuffError", "build_codebook", "encoded_bits", "dcb_to_host", "load", "DCB_BYTES"]

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


def _struct_dtype(cls) -> np.dtype:
    """numpy dtype with the field offsets and size of a ctypes struct."""
    kinds = {ctypes.c_int32: "<i4", ctypes.c_uint32: "<u4", ctypes.c_uint64: "<u8", ctypes.c_void_p: "<u8",
             ctypes.c_double: "<f8"}
    names = [f for f, _ in cls._fields_]
    return np.dtype({"names": names, "formats": [kinds[t] for _, t in cls._fields_],
                     "offsets": [getattr(cls, f).offset for f in names], "itemsize": ctypes.sizeof(cls)})


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

    def set_timing(self, enable: bool = True):
        """huff_ctx_set_timing: record HIP events around this context's kernel
        launches (single-stream calls only)."""
        _check(lib().huff_ctx_set_timing(self._ctx, 1 if enable else 0), "huff_ctx_set_timing")

    def kernel_time(self, kernel: str, reset: bool = True) -> tuple[float, int]:
        """huff_ctx_kernel_time: (summed launch ms, launches) of one kernel
        ('hist', 'codebook', 'scan', 'encode' or 'decode')."""
        ms, k = ctypes.c_double(), ctypes.c_uint64()
        _check(lib().huff_ctx_kernel_time(self._ctx, _abi.KERNEL_IDS[kernel], ctypes.byref(ms), ctypes.byref(k),
                                          1 if reset else 0), "huff_ctx_kernel_time")
        return float(ms.value), int(k.value)

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

    # -- Method 3: block transform before the Huffman code --------------------
    def bwt(self, x, block: int, every: int, last=None, rows=None, stream=None):
        """huff_bwt: (last column uint8[n], rows int16 view of u16[ceil(n/every)])."""
        torch = _torch()
        x = self._u8(x)
        n = x.numel()
        if last is None:
            last = torch.empty(n, dtype=torch.uint8, device=self.device)
        if rows is None:
            rows = torch.empty(max(1, (n + every - 1) // every), dtype=torch.int16, device=self.device)
        _check(lib().huff_bwt(self._ctx, _ptr(x), n, block, every, _ptr(last), _ptr(rows), self._stream(stream)),
               "huff_bwt")
        return last, rows

    def unbwt(self, last, block: int, every: int, rows, out=None, status=None, stream=None):
        torch = _torch()
        last = self._u8(last)
        n = last.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().huff_unbwt(self._ctx, _ptr(last), n, block, every, _ptr(rows), _ptr(out), _ptr(status),
                                self._stream(stream)), "huff_unbwt")
        return out

    def mtf(self, x, block: int, out=None, stream=None):
        torch = _torch()
        x = self._u8(x)
        if out is None:
            out = torch.empty(x.numel(), dtype=torch.uint8, device=self.device)
        _check(lib().huff_mtf(self._ctx, _ptr(x), x.numel(), block, _ptr(out), self._stream(stream)), "huff_mtf")
        return out

    def unmtf(self, x, block: int, out=None, stream=None):
        torch = _torch()
        x = self._u8(x)
        if out is None:
            out = torch.empty(x.numel(), dtype=torch.uint8, device=self.device)
        _check(lib().huff_unmtf(self._ctx, _ptr(x), x.numel(), block, _ptr(out), self._stream(stream)), "huff_unmtf")
        return out

    def compress_bwt(self, x, block: int, every: int, chunk_size: int, sub_size: int = 0, status=None, stream=None,
                     out: dict | None = None) -> dict:
        """Method 3: huff_bwt, huff_mtf, then huff_compress of the positions.
        `out` may hold preallocated last/rows/mtf tensors and huff_compress's."""
        o = dict(out or {})
        last, rows = self.bwt(x, block, every, last=o.get("last"), rows=o.get("rows"), stream=stream)
        m = self.mtf(last, block, out=o.get("mtf"), stream=stream)
        c = self.compress(m, chunk_size, sub_size, status=status, stream=stream, out=o)
        c.update(last=last, rows=rows, mtf=m, block=block, every=every)
        return c

    def decompress_bwt(self, c: dict, out=None, status=None, stream=None, work: dict | None = None):
        """Inverse of compress_bwt: huff_decode, huff_unmtf, huff_unbwt."""
        w = dict(work or {})
        m = self.decompress(c, out=w.get("mtf"), status=status, stream=stream)
        last = self.unmtf(m, c["block"], out=w.get("last"), stream=stream)
        return self.unbwt(last, c["block"], c["every"], c["rows"], out=out, status=status, stream=stream)

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

    def compress_noalloc(self, x, chunk_size: int, sub_size: int, out: dict, status=None, stream=None) -> dict:
        """huff_compress_noalloc: huff_compress with the library's fixed device
        workspace (no allocation by the library; at most HUFF_NOALLOC_MAX_N
        bytes).  `out` must hold preallocated hist/dcb/words/chunk_off (and
        sub_lo when sub_size) tensors."""
        x = self._u8(x)
        n = x.numel()
        words = out["words"]
        _check(lib().huff_compress_noalloc(self._ctx, _ptr(x), n, chunk_size, _ptr(out["dcb"]), _ptr(out.get("hist")),
                                           _ptr(words), words.numel(), _ptr(out["chunk_off"]), sub_size,
                                           _ptr(out.get("sub_lo")) if sub_size else None, _ptr(status),
                                           self._stream(stream)), "huff_compress_noalloc")
        return dict(hist=out.get("hist"), dcb=out["dcb"], words=words, chunk_off=out["chunk_off"],
                    sub_lo=out.get("sub_lo") if sub_size else None, n=n, chunk_size=chunk_size, sub_size=sub_size)

    def decompress(self, c: dict, out=None, status=None, stream=None):
        return self.decode(c["words"], c["words"].numel(), c["chunk_off"], c["n"], c["chunk_size"], c["dcb"],
                           c.get("sub_lo"), c.get("sub_size", 0), out=out, status=status, stream=stream)


class Batch:
    """A batch plan (``huff_batch``): many files, each with its own codebook,
    handled by one fixed sequence of launches per operation.

    ``files`` is a list of dicts of device tensors: ``in`` (uint8, n bytes),
    ``cb`` (DCB_BYTES), ``words`` (int32 view of u32), ``chunk_off`` (int64),
    optionally ``sub_lo`` (int32), ``out`` (uint8), ``hist`` (int64, 256),
    ``status`` (int32, 1).  Tensors are referenced, not copied: keep them
    alive and in place while the batch is used (a captured graph replays the
    same addresses).
    """

    def __init__(self, codec: "Codec", files: list, chunk_size: int, sub_size: int = 0):
        self.codec = codec
        self.files = files
        self.chunk_size, self.sub_size = chunk_size, sub_size
        arr = (HuffFile * max(1, len(files)))()
        for i, f in enumerate(files):
            x = f.get("in")
            n = int(f["n"]) if "n" in f else int(x.numel())
            arr[i] = HuffFile(_ptr(x), n, _ptr(f["cb"]), _ptr(f.get("words")),
                              0 if f.get("words") is None else f["words"].numel(), _ptr(f["chunk_off"]),
                              _ptr(f.get("sub_lo")), _ptr(f.get("out")), _ptr(f.get("hist")), _ptr(f.get("status")))
        h = ctypes.c_void_p()
        _check(lib().huff_batch_create(codec._ctx, arr, len(files), chunk_size, sub_size, ctypes.byref(h)),
               "huff_batch_create")
        self._h = h

    def run(self, op: int, graph: bool = False, stream=None):
        _check(lib().huff_batch_run(self._h, op, int(graph), self.codec._stream(stream)), "huff_batch_run")

    def compress(self, graph: bool = False, stream=None):
        self.run(HUFF_OP_COMPRESS, graph, stream)

    def encode(self, graph: bool = False, stream=None):
        self.run(HUFF_OP_ENCODE, graph, stream)

    def decode(self, graph: bool = False, stream=None):
        self.run(HUFF_OP_DECODE, graph, stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().huff_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_buffers(codec: "Codec", inputs: list, chunk_size: int, sub_size: int = 0, decode: bool = True,
                  bits_per_byte: int = 16) -> list:
    """Allocates per-file output tensors for a batch over the device uint8
    tensors `inputs`.  The word capacity holds `bits_per_byte` bits per input
    byte (16 covers every codebook whose longest code has at most 16 bits; a
    file that needs more reports HUFF_E_CAPACITY in its status word)."""
    torch = _torch()
    dev = codec.device
    files = []
    for x in inputs:
        n = x.numel()
        nch = (n + chunk_size - 1) // chunk_size
        f = {"in": x, "n": n,
             "cb": torch.empty(DCB_BYTES, dtype=torch.uint8, device=dev),
             "words": torch.empty((n * bits_per_byte + 31) // 32 + 8, dtype=torch.int32, device=dev),
             "chunk_off": torch.empty(nch + 1, dtype=torch.int64, device=dev),
             "hist": torch.empty(256, dtype=torch.int64, device=dev),
             "status": torch.zeros(1, dtype=torch.int32, device=dev)}
        if sub_size:
            f["sub_lo"] = torch.empty((n + sub_size - 1) // sub_size + 1, dtype=torch.int32, device=dev)
        if decode:
            f["out"] = torch.empty(n, dtype=torch.uint8, device=dev)
        files.append(f)
    return files


class Segments:
    """Per-segment codebooks within one stream (Method 2 as the paper states
    it: the input cut into segments, each coded with a tree of its own, the
    coded segments kept in segment order).  One batch plan over the segments
    does the work; its outputs live in single allocations, one fixed-size
    region per segment: ``cb`` [nseg, DCB_BYTES], ``words`` [nseg, wcap],
    ``chunk_off`` [nseg, nch + 1], ``sub_lo`` [nseg, nsub + 1], ``hist``
    [nseg, 256], ``status`` [nseg] and ``out`` (n bytes, decode output).
    Chunks and sub-blocks restart at every segment.  ``seg_size`` is a
    multiple of 16 so that every segment of a 16-byte aligned input is too.
    """

    def __init__(self, codec: "Codec", x, seg_size: int, chunk_size: int, sub_size: int = 0, decode: bool = True):
        torch = _torch()
        if seg_size <= 0 or seg_size % 16:
            raise ValueError("seg_size must be a positive multiple of 16")
        x = codec._u8(x)
        n = x.numel()
        dev = codec.device
        self.n, self.seg_size = n, seg_size
        self.nseg = nseg = (n + seg_size - 1) // seg_size
        nch = (seg_size + chunk_size - 1) // chunk_size
        wcap = ((seg_size * 16 + 31) // 32 + 8 + 3) // 4 * 4  # 16 bits per byte, 16-byte rows
        self.cb = torch.empty((max(1, nseg), DCB_BYTES), dtype=torch.uint8, device=dev)
        self.words = torch.empty((max(1, nseg), wcap), dtype=torch.int32, device=dev)
        self.chunk_off = torch.empty((max(1, nseg), nch + 1), dtype=torch.int64, device=dev)
        self.sub_lo = None
        if sub_size:
            nsub = (seg_size + sub_size - 1) // sub_size
            self.sub_lo = torch.empty((max(1, nseg), nsub + 1), dtype=torch.int32, device=dev)
        self.hist = torch.empty((max(1, nseg), 256), dtype=torch.int64, device=dev)
        self.status = torch.zeros(max(1, nseg), dtype=torch.int32, device=dev)
        self.out = torch.empty(n, dtype=torch.uint8, device=dev) if decode else None
        files = []
        for i in range(nseg):
            lo, hi = i * seg_size, min(n, (i + 1) * seg_size)
            f = {"in": x[lo:hi], "n": hi - lo, "cb": self.cb[i], "words": self.words[i],
                 "chunk_off": self.chunk_off[i, :(hi - lo + chunk_size - 1) // chunk_size + 1],
                 "hist": self.hist[i], "status": self.status[i:i + 1]}
            if sub_size:
                f["sub_lo"] = self.sub_lo[i, :(hi - lo + sub_size - 1) // sub_size + 1]
            if decode:
                f["out"] = self.out[lo:hi]
            files.append(f)
        self.files = files
        self.batch = Batch(codec, files, chunk_size, sub_size)

    def compress(self, graph: bool = False, stream=None):
        self.batch.compress(graph, stream)

    def decode(self, graph: bool = False, stream=None):
        self.batch.decode(graph, stream)

    def segment_bits(self):
        """Code bits of every segment: the last entry of its segment index (one copy to the host)."""
        off = self.chunk_off.cpu()
        return [int(off[i, f["chunk_off"].numel() - 1]) for i, f in enumerate(self.files)]

    def close(self):
        self.batch.close()


class Server:
    """The request server (``huff_server``) on a context of its own.

    ``submit_compress(x)`` / ``submit_decode(handle)`` queue requests and
    return tickets; ``wait(ticket)`` / ``poll(ticket)`` give result dicts;
    ``stream(handle)`` gives device pointers of a resident stream or decode
    output; ``release(handle)`` frees it; ``replay(...)`` drives an open-loop
    arrival schedule natively."""

    def __init__(self, device: int = 0, mem_budget: int = 1 << 30, nslots: int = 2, max_batch: int = 512,
                 chunk_size: int = 256 << 10, sub_size: int = 0, params: dict | None = None):
        self.codec = Codec(device, params)  # the server takes this context over
        cfg = HuffServerCfg(mem_budget, nslots, max_batch, chunk_size, sub_size)
        h = ctypes.c_void_p()
        _check(lib().huff_server_create(self.codec._ctx, ctypes.byref(cfg), ctypes.byref(h)), "huff_server_create")
        self._h = h
        self.chunk_size, self.sub_size = chunk_size, sub_size
        self._keep = {}  # ticket -> input tensor, alive until the request is done

    @staticmethod
    def _res(r: HuffResult) -> dict:
        return {k: getattr(r, k) for k, _ in HuffResult._fields_}

    def submit_compress(self, x, expect=None, expect_bits: int = 0) -> int:
        """Queues a compress of x.  With `expect` (device tensor of the
        expected stream words) and `expect_bits` (expected T), the server
        compares the result on the device (status HUFF_E_MISMATCH if it
        differs)."""
        t = ctypes.c_uint64()
        req = HuffRequest(HUFF_OP_COMPRESS, 0, _ptr(x), x.numel(), 0, _ptr(expect), expect_bits)
        _check(lib().huff_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "huff_server_submit")
        self._keep[t.value] = (x, expect)
        return t.value

    def submit_decode(self, handle: int, expect=None) -> int:
        """Queues a decode of a resident stream; with `expect` (device tensor
        of the expected bytes) the result is compared on the device."""
        t = ctypes.c_uint64()
        req = HuffRequest(HUFF_OP_DECODE, 0, None, 0, handle, _ptr(expect), 0)
        _check(lib().huff_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "huff_server_submit")
        self._keep[t.value] = (None, expect)
        return t.value

    def wait(self, ticket: int) -> dict:
        r = HuffResult()
        _check(lib().huff_server_wait(self._h, ticket, ctypes.byref(r)), "huff_server_wait")
        self._keep.pop(ticket, None)
        return self._res(r)

    def poll(self, ticket: int):
        r = HuffResult()
        rc = lib().huff_server_poll(self._h, ticket, ctypes.byref(r))
        if rc == HUFF_E_AGAIN:
            return None
        _check(rc, "huff_server_poll")
        self._keep.pop(ticket, None)
        return self._res(r)

    def stream(self, handle: int) -> dict:
        i = HuffStreamInfo()
        _check(lib().huff_server_stream(self._h, handle, ctypes.byref(i)), "huff_server_stream")
        return {k: getattr(i, k) for k, _ in HuffStreamInfo._fields_}

    def release(self, handle: int):
        _check(lib().huff_server_release(self._h, handle), "huff_server_release")

    def replay(self, requests: list, arrivals, discard=None) -> list:
        """requests: list of (op, tensor_or_None, handle) or (op, tensor_or_None,
        handle, expect_ptr, expect_bits) (an expected result, compared on the
        device); arrivals: seconds; discard: indexes whose results are freed as
        soon as they are done (True: all)."""
        n = len(requests)
        reqs = (HuffRequest * max(1, n))()
        drop = discard if discard is True else set(discard or ())
        for i, rq in enumerate(requests):
            op, x, h = rq[0], rq[1], rq[2]
            ep, eb = (rq[3], rq[4]) if len(rq) > 3 else (None, 0)
            reqs[i] = HuffRequest(op, 1 if (drop is True or i in drop) else 0, _ptr(x), 0 if x is None else x.numel(),
                                  h or 0, ep, eb)
        arr = np.ascontiguousarray(arrivals, dtype=np.float64)
        res = (HuffResult * max(1, n))()
        _check(lib().huff_server_replay(self._h, reqs, arr.ctypes.data, n, res), "huff_server_replay")
        return [self._res(res[i]) for i in range(n)]

    @staticmethod
    def request_array(count: int) -> np.ndarray:
        """A zeroed numpy array laid out as `count` huff_request structs
        (fields op, flags, d_in, n, stream_handle, d_expect, expect_bits)."""
        return np.zeros(count, dtype=_struct_dtype(HuffRequest))

    def replay_array(self, reqs: np.ndarray, arrivals) -> np.ndarray:
        """huff_server_replay over a request_array(); returns the results as a
        numpy array laid out as huff_result structs.  Keep the tensors the
        requests point to alive until this returns."""
        reqs = np.ascontiguousarray(reqs, dtype=_struct_dtype(HuffRequest))
        arr = np.ascontiguousarray(arrivals, dtype=np.float64)
        assert arr.size == reqs.size
        res = np.zeros(max(1, reqs.size), dtype=_struct_dtype(HuffResult))
        _check(lib().huff_server_replay(self._h, reqs.ctypes.data, arr.ctypes.data, reqs.size, res.ctypes.data),
               "huff_server_replay")
        return res[:reqs.size]

    def stats(self) -> dict:
        a = (ctypes.c_uint64 * 6)()
        _check(lib().huff_server_stats(self._h, a), "huff_server_stats")
        return dict(zip(("batches", "done", "mem_used", "mem_peak", "waiting", "inflight"), list(a)))

    def close(self):
        if getattr(self, "_h", None):
            lib().huff_server_destroy(self._h)
            self._h = None
            self.codec.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
