"""CPU oracle for the Huffman codec -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports or calls it.

It wraps ``oracle.c`` (plain serial C, built with gcc by ``build()``), which
follows Section III.A of the paper (Method 1: frequency count, repeated
merging of the two lowest-weight nodes into one whose weight is their sum;
Method 2: segments reassembled by id).  The readings of points the paper
leaves open are stated at the top of ``oracle.c``: (weight, id) tie rule,
canonical codes, MSB-first 32-bit words, bit-contiguous chunks with a u64
bit-offset index.

Parity status of each function against pins that do not come from the oracle
itself (see ``tests/test_oracle.py``):
  histogram          pinned: numpy.bincount
  code_lengths       pinned: brute-force optimal cost (K <= 7), closed forms
                     (uniform, dyadic, Fibonacci), textbook example, Kraft
                     equality, entropy bound.  The tie-specific choice among
                     optimal codes is fixed by the stated rule and checked by a
                     second, independent implementation (two-queue).
  canonical_codes    pinned: RFC 1951 worked example, hand-derived example
  encode             pinned: hand-derived bitstream, string-concatenation
                     re-encoding, T = sum(h*len), chunk independence
  decode             pinned: round trip, corruption cases
  bwt / unbwt        pinned: the Burrows-Wheeler worked examples (tests/golden),
                     brute-force sorted rotations on small blocks, inverse
                     round trip, permutation of each block
  mtf / unmtf        pinned: a worked example from the standard description
                     (tests/golden), runs give zeros, round trip
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, INVAL, CAPACITY, CORRUPT, CODELEN = 0, -1, -2, -3, -7


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build() -> str:
    """Compile the oracle library in place (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC,
                           os.path.join(_HERE, "bwt.c")])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    lib.oracle_histogram.argtypes = [vp, u64, vp]
    lib.oracle_code_lengths.argtypes = [vp, vp]
    lib.oracle_code_lengths_twoqueue.argtypes = [vp, vp]
    lib.oracle_canonical_codes.argtypes = [vp, vp]
    lib.oracle_total_bits.argtypes = [vp, vp]
    lib.oracle_total_bits.restype = u64
    lib.oracle_encode.argtypes = [vp, u64, vp, vp, u64, vp, u64, vp]
    lib.oracle_decode.argtypes = [vp, u64, vp, u64, u64, vp, vp]
    u32 = ctypes.c_uint32
    lib.oracle_bwt.argtypes = [vp, u64, u32, u32, vp, vp]
    lib.oracle_unbwt.argtypes = [vp, u64, u32, u32, vp, vp]
    lib.oracle_mtf.argtypes = [vp, u64, u32, vp]
    lib.oracle_unmtf.argtypes = [vp, u64, u32, vp]
    for f in ("oracle_histogram", "oracle_code_lengths", "oracle_code_lengths_twoqueue",
              "oracle_canonical_codes", "oracle_encode", "oracle_decode", "oracle_bwt", "oracle_unbwt",
              "oracle_mtf", "oracle_unmtf"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data if a.size else None


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


def histogram(data) -> np.ndarray:
    a = _u8(data)
    h = np.zeros(256, dtype=np.uint64)
    _check(_load().oracle_histogram(_p(a), a.size, h.ctypes.data), "histogram")
    return h


def code_lengths(hist, method: str = "heap") -> np.ndarray:
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    assert h.size == 256
    ln = np.zeros(256, dtype=np.uint8)
    fn = _load().oracle_code_lengths if method == "heap" else _load().oracle_code_lengths_twoqueue
    _check(fn(h.ctypes.data, ln.ctypes.data), "code_lengths")
    return ln


def canonical_codes(lengths) -> np.ndarray:
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    code = np.zeros(256, dtype=np.uint64)
    _check(_load().oracle_canonical_codes(ln.ctypes.data, code.ctypes.data), "canonical_codes")
    return code


def total_bits(hist, lengths) -> int:
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    return int(_load().oracle_total_bits(h.ctypes.data, ln.ctypes.data))


def encode(data, lengths, codes, chunk: int):
    """Returns (words u32[ceil(T/32)], chunk_off u64[ceil(n/chunk)+1])."""
    a = _u8(data)
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    cd = np.ascontiguousarray(codes, dtype=np.uint64)
    t = int(np.sum(ln[a].astype(np.uint64))) if a.size else 0
    words = np.zeros(max(1, (t + 31) // 32), dtype=np.uint32)
    off = np.zeros((a.size + chunk - 1) // chunk + 1, dtype=np.uint64)
    _check(_load().oracle_encode(_p(a), a.size, ln.ctypes.data, cd.ctypes.data, chunk, words.ctypes.data,
                                 (t + 31) // 32, off.ctypes.data), "encode")
    return words[: (t + 31) // 32], off


def decode(words, chunk_off, n: int, chunk: int, lengths) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint32)
    off = np.ascontiguousarray(chunk_off, dtype=np.uint64)
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    out = np.zeros(n, dtype=np.uint8)
    _check(_load().oracle_decode(_p(w), w.size, off.ctypes.data, n, chunk, ln.ctypes.data, _p(out)), "decode")
    return out


def sub_index(chunk_off_fine) -> np.ndarray:
    """Low 32 bits of the bit offsets at a fine granularity (the decode index)."""
    return (np.asarray(chunk_off_fine, dtype=np.uint64) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def compress(data, chunk: int, sub: int | None = None) -> dict:
    """Whole oracle pipeline: histogram, lengths, canonical codes, encode.
    With ``sub``, also the decode index (offsets every ``sub`` bytes, low 32 bits)."""
    a = _u8(data)
    h = histogram(a)
    ln = code_lengths(h)
    cd = canonical_codes(ln)
    words, off = encode(a, ln, cd, chunk)
    out = dict(hist=h, len=ln, code=cd, words=words, chunk_off=off, total_bits=int(off[-1]))
    if sub is not None:
        if sub == chunk:
            out["sub_lo"] = sub_index(off)
        else:
            _, fine = encode(a, ln, cd, sub)
            out["sub_lo"] = sub_index(fine)
    return out


# ---- Method 3: block transform before the Huffman code (oracle/bwt.c) ----
def bwt(data, block: int, every: int):
    """Burrows-Wheeler transform block by block.  Returns (last, rows):
    last[i] the last-column byte, rows[j] the sorted row of the rotation that
    starts at byte j*every (within its block); rows has ceil(n/every) entries
    and rows[b*block/every] is block b's primary index."""
    a = _u8(data)
    last = np.zeros(a.size, dtype=np.uint8)
    rows = np.zeros((a.size + every - 1) // every, dtype=np.uint32)
    _check(_load().oracle_bwt(_p(a), a.size, block, every, _p(last), _p(rows)), "bwt")
    return last, rows


def unbwt(last, block: int, every: int, rows) -> np.ndarray:
    a = _u8(last)
    r = np.ascontiguousarray(rows, dtype=np.uint32)
    out = np.zeros(a.size, dtype=np.uint8)
    _check(_load().oracle_unbwt(_p(a), a.size, block, every, _p(r), _p(out)), "unbwt")
    return out


def mtf(data, block: int) -> np.ndarray:
    """Move-to-front positions, the list (byte values in order) reset every `block` bytes."""
    a = _u8(data)
    out = np.zeros(a.size, dtype=np.uint8)
    _check(_load().oracle_mtf(_p(a), a.size, block, _p(out)), "mtf")
    return out


def unmtf(data, block: int) -> np.ndarray:
    a = _u8(data)
    out = np.zeros(a.size, dtype=np.uint8)
    _check(_load().oracle_unmtf(_p(a), a.size, block, _p(out)), "unmtf")
    return out


def compress_bwt(data, block: int, every: int, chunk: int, sub: int | None = None) -> dict:
    """Method 3: block transform, move-to-front, then Method 1's Huffman code
    over the whole transformed stream (chunk index as Method 2's segment ids)."""
    last, rows = bwt(data, block, every)
    m = mtf(last, block)
    out = compress(m, chunk, sub)
    out.update(last=last, rows=rows, mtf=m)
    return out
