"""Seeded synthetic byte streams shared by the oracle tests, the GPU tests and
the benchmark.  This module only draws input bytes; it holds none of the
codec's arithmetic.

The paper evaluates Huffman coding on a 45 MB English book corpus
(Section III.A).  That corpus is not available, so these generators stand in
for it (order-2 Markov text over the 96 printable symbols, word-level text
from a seeded Zipf vocabulary, and i.i.d. Zipf bytes).  The C source is
``gen.c``; ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libhuffgen.so")
_lib = None

#: The 96 printable symbols in their fixed base order: newline, then 0x20..0x7E.
A96 = np.array([0x0A] + list(range(0x20, 0x7F)), dtype=np.uint8)
#: All 256 byte values.
A256 = np.arange(256, dtype=np.uint8)


def build() -> str:
    """Compile the generator library in place (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.gen_block_bytes.restype = ctypes.c_uint32
    lib.gen_permutation.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u8p]
    lib.gen_zipf_iid.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, u8p,
                                 ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]
    lib.gen_zipf_iid.restype = ctypes.c_int
    lib.gen_markov_table_bytes.restype = ctypes.c_uint32
    lib.gen_markov_table.argtypes = [ctypes.c_uint64, u8p]
    lib.gen_markov.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, u8p, ctypes.c_uint64, ctypes.c_uint64]
    lib.gen_markov.restype = ctypes.c_int
    lib.gen_words_scratch_bytes.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.gen_words_scratch_bytes.restype = ctypes.c_uint64
    lib.gen_words_vocab.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
    lib.gen_words_vocab.restype = ctypes.c_int
    lib.gen_words.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32,
                              ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_uint64,
                              ctypes.c_uint64]
    lib.gen_words.restype = ctypes.c_int
    lib.gen_file_params.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_uint32)]
    _lib = lib
    return lib


def _u8p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _out(n: int, out):
    if out is None:
        return np.empty(n, dtype=np.uint8)
    assert out.dtype == np.uint8 and out.flags.c_contiguous and out.size >= n
    return out[:n]


def permutation(symbols: np.ndarray, seed: int, stream: int = 0) -> np.ndarray:
    """Seeded Fisher-Yates permutation of ``symbols`` (rank order of a Zipf draw)."""
    lib = _load()
    sym = np.ascontiguousarray(symbols, dtype=np.uint8)
    out = np.empty_like(sym)
    lib.gen_permutation(_u8p(sym), sym.size, seed, stream, _u8p(out))
    return out


def _blocks(n: int, fn):
    lib = _load()
    blk = lib.gen_block_bytes()
    nblk = (n + blk - 1) // blk
    if nblk <= 1:
        fn(0, nblk)
        return
    w = min(_workers(), nblk)
    step = (nblk + w - 1) // w
    with ThreadPoolExecutor(w) as ex:
        list(ex.map(lambda lo: fn(lo, min(nblk, lo + step)), range(0, nblk, step)))


def zipf_iid(n: int, seed: int, s: float, symbols: np.ndarray = A96, k: int | None = None, out=None) -> np.ndarray:
    """n i.i.d. bytes, Zipf(s) over the first ``k`` entries of a seeded
    permutation of ``symbols`` (rank 1 = the first of them)."""
    lib = _load()
    k = len(symbols) if k is None else k
    alpha = np.ascontiguousarray(permutation(symbols, seed, 1)[:k])
    buf = _out(n, out)
    ptr = buf.ctypes.data

    def run(lo, hi):
        rc = lib.gen_zipf_iid(ptr, n, seed, s, _u8p(alpha), k, lo, hi)
        assert rc == 0

    _blocks(n, run)
    return buf


_tables: dict[int, np.ndarray] = {}


def markov_table(seed: int) -> np.ndarray:
    if seed not in _tables:
        lib = _load()
        t = np.empty(lib.gen_markov_table_bytes(), dtype=np.uint8)
        lib.gen_markov_table(seed, _u8p(t))
        _tables[seed] = t
    return _tables[seed]


def markov(n: int, seed: int, s: float = 1.0, line_mu: float = 70.0, line_sigma: float = 15.0, out=None) -> np.ndarray:
    """n bytes of order-2 Markov text over the 96 printable symbols."""
    lib = _load()
    table = markov_table(seed)
    buf = _out(n, out)
    ptr = buf.ctypes.data

    def run(lo, hi):
        rc = lib.gen_markov(ptr, n, seed, s, line_mu, line_sigma, _u8p(table), lo, hi)
        assert rc == 0

    _blocks(n, run)
    return buf


def words(n: int, seed: int, s: float = 1.0, vocab: int = 8192, max_word: int = 8, line_mu: float = 70.0,
          line_sigma: float = 15.0, out=None) -> np.ndarray:
    """n bytes of word-level text: words drawn i.i.d. Zipf(s) from a seeded
    vocabulary of lowercase words, separated by spaces, lines broken after
    about N(70, 15) characters."""
    lib = _load()
    scratch = np.empty(lib.gen_words_scratch_bytes(vocab, max_word), dtype=np.uint8)
    assert lib.gen_words_vocab(seed, vocab, max_word, scratch.ctypes.data) == 0
    buf = _out(n, out)
    ptr = buf.ctypes.data

    def run(lo, hi):
        rc = lib.gen_words(ptr, n, seed, s, vocab, max_word, line_mu, line_sigma, scratch.ctypes.data, lo, hi)
        assert rc == 0

    _blocks(n, run)
    return buf


def file_params(seed: int, i: int, size_lo: int = 4096, size_hi: int = 1 << 24, s_lo: float = 0.6,
                s_hi: float = 1.6, k_lo: int = 16, k_hi: int = 256):
    """(size, zipf exponent, alphabet size) of file ``i`` of a batched set."""
    lib = _load()
    size, s, k = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_uint32()
    lib.gen_file_params(seed, i, size_lo, size_hi, s_lo, s_hi, k_lo, k_hi, ctypes.byref(size), ctypes.byref(s),
                        ctypes.byref(k))
    return int(size.value), float(s.value), int(k.value)


def batch_file(seed: int, i: int, out=None, **kw) -> np.ndarray:
    """File ``i`` of the batched set: i.i.d. Zipf bytes over the first K of a
    seeded permutation of all 256 byte values."""
    size, s, k = file_params(seed, i, **kw)
    return zipf_iid(size, seed * 1_000_003 + i + 1, s, A256, k, out=out)


# Named workloads (sizes and seeds).  cfg1: 1 MiB Zipf(1.1)/96; cfg2: 45 MiB
# Markov text; cfg3a: 2 GiB Markov text; cfg3b: 2 GiB Zipf(0.8)/256;
# cfg4: 4096 files; serving requests draw Markov text with their own seeds.
WORKLOADS = {
    "zipf96_1MiB": dict(n=1 << 20, chunk=64 << 10),
    "markov_45MiB": dict(n=45 << 20, chunk=256 << 10),
    "markov_2GiB": dict(n=1 << 31, chunk=None),
    "zipf256_2GiB": dict(n=1 << 31, chunk=None),
    "markov_1GiB": dict(n=1 << 30, chunk=None),   # the leading 2^30 bytes of markov_2GiB
    "zipf256_1GiB": dict(n=1 << 30, chunk=None),  # the leading 2^30 bytes of zipf256_2GiB
    "words_45MiB": dict(n=45 << 20, chunk=256 << 10),  # word-level text, the block transform's workload
    "words_1GiB": dict(n=1 << 30, chunk=None),
}


def workload(name: str, n: int | None = None, out=None) -> np.ndarray:
    """Bytes of a named workload; ``n`` truncates it (same leading bytes)."""
    full = WORKLOADS[name]["n"]
    n = full if n is None else n
    if name == "zipf96_1MiB":
        return zipf_iid(n, 1, 1.1, A96, out=out)
    if name == "markov_45MiB":
        return markov(n, 2, out=out)
    if name in ("markov_2GiB", "markov_1GiB"):
        return markov(n, 3, out=out)
    if name in ("zipf256_2GiB", "zipf256_1GiB"):
        return zipf_iid(n, 4, 0.8, A256, out=out)
    if name in ("words_45MiB", "words_1GiB"):
        return words(n, 7, out=out)
    raise KeyError(name)
