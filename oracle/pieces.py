"""Whole-stream parity of a long stream against the CPU oracle -- TEST
INFRASTRUCTURE ONLY (loaded by the tests and the benchmark's oracle legs).

The oracle encodes the input piece by piece (each piece a whole number of
chunks and sub-blocks) in a thread pool; its C calls release the GIL, so the
pieces run in parallel.  Every piece's code bits are compared with the GPU
words at the bit where the GPU's segment index says the piece starts, and the
piece starts are then checked against the running sum of the oracle's piece
totals, so that together the comparisons cover every word, every chunk offset
and every sub-block offset of the stream (Section III.A, Method 2: the coded
segments put back together in id order are the coded stream).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import encode as _encode

_M32 = np.uint64(0xFFFFFFFF)


def bits_equal(g_words: np.ndarray, b0: int, w: np.ndarray, t: int, last: bool) -> bool:
    """Stream bits [b0, b0 + t) of the u32 words `g_words` equal bits [0, t)
    of `w`.  With `last`, the unused bits after the stream's final bit must
    be zero in `g_words` too (the oracle's are)."""
    if t == 0:
        return True
    s = b0 & 31
    w0 = b0 >> 5
    wl = w[: (t + 31) // 32].astype(np.uint64)
    if s:
        prev = np.concatenate((np.zeros(1, np.uint64), wl))
        cur = np.concatenate((wl, np.zeros(1, np.uint64)))
        shifted = ((prev << np.uint64(32)) | cur) >> np.uint64(s) & _M32
    else:
        shifted = wl
    ns = (s + t + 31) // 32
    shifted = shifted[:ns]
    g = g_words[w0:w0 + ns].astype(np.uint64)
    if g.size != ns:
        return False
    mask = np.full(ns, 0xFFFFFFFF, dtype=np.uint64)
    mask[0] &= np.uint64(0xFFFFFFFF >> s)
    end = (s + t) & 31
    if end and not last:
        mask[-1] &= np.uint64((0xFFFFFFFF << (32 - end)) & 0xFFFFFFFF)
    return bool(np.array_equal(g & mask, shifted & mask))


def check_stream(a: np.ndarray, words: np.ndarray, chunk_off: np.ndarray, sub_lo, lengths, codes, chunk: int,
                 sub: int, piece: int = 8 << 20, workers: int | None = None) -> int:
    """Asserts that (words, chunk_off, sub_lo) is exactly the oracle's stream
    of `a` under the code (lengths, codes).  Returns T, the total bits."""
    n = a.size
    step = max(chunk, sub or 1)
    piece = max(step, piece // step * step)
    npieces = (n + piece - 1) // piece
    workers = workers or max(1, min(16, os.cpu_count() or 1))

    def one(p):
        lo, hi = p * piece, min(n, (p + 1) * piece)
        seg = a[lo:hi]
        w, off = _encode(seg, lengths, codes, chunk)
        t = int(off[-1])
        c0 = lo // chunk
        b0 = int(chunk_off[c0])
        ok_off = np.array_equal(chunk_off[c0:c0 + off.size].astype(np.uint64), off + np.uint64(b0))
        ok_sub = True
        if sub:
            _, fine = _encode(seg, lengths, codes, sub)
            s0 = lo // sub
            want = (fine + np.uint64(b0)) & _M32
            ok_sub = np.array_equal(sub_lo[s0:s0 + fine.size].astype(np.uint64), want)
        ok_bits = bits_equal(words, b0, w, t, last=(hi == n))
        return p, b0, t, ok_off, ok_sub, ok_bits

    with ThreadPoolExecutor(workers) as ex:
        res = sorted(ex.map(one, range(npieces)))
    run = 0
    for p, b0, t, ok_off, ok_sub, ok_bits in res:
        assert b0 == run, f"piece {p}: segment index starts at bit {b0}, oracle {run}"
        assert ok_off, f"piece {p}: chunk offsets differ from the oracle"
        assert ok_sub, f"piece {p}: sub-block offsets differ from the oracle"
        assert ok_bits, f"piece {p}: words differ from the oracle"
        run += t
    assert int(chunk_off[-1]) == run
    if n:
        assert chunk_off.size == (n + chunk - 1) // chunk + 1
    return run
