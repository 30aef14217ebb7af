"""The piecewise whole-stream checker (oracle/pieces.py) accepts the
oracle's own stream and rejects any single changed bit, offset or index
entry (CPU only)."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import pieces as oracle_pieces


@pytest.fixture(scope="module")
def stream():
    a = datagen.markov(3 * (1 << 20) + 777, 41)
    chunk, sub = 64 << 10, 256
    r = oracle.compress(a, chunk, sub=sub)
    return a, chunk, sub, r


def _check(a, chunk, sub, r, words=None, off=None, sub_lo=None):
    return oracle_pieces.check_stream(a, r["words"] if words is None else words,
                                      r["chunk_off"] if off is None else off,
                                      r["sub_lo"] if sub_lo is None else sub_lo,
                                      r["len"], r["code"], chunk, sub, piece=1 << 20, workers=4)


def test_accepts_the_oracle_stream(stream):
    a, chunk, sub, r = stream
    assert _check(a, chunk, sub, r) == r["total_bits"]


@pytest.mark.parametrize("bit", [0, 31, 32 * 1000 + 7, None])
def test_rejects_a_flipped_word_bit(stream, bit):
    a, chunk, sub, r = stream
    w = r["words"].copy()
    t = r["total_bits"]
    if bit is None:  # an unused trailing bit of the last word must stay zero
        assert t % 32, "the fixture must leave unused bits"
        bit = t  # first unused bit
    if bit == 32 * 1000 + 7:
        bit = int(r["chunk_off"][20]) + 5  # inside a later piece
    w[bit // 32] ^= np.uint32(1 << (31 - bit % 32))
    with pytest.raises(AssertionError):
        _check(a, chunk, sub, r, words=w)


def test_rejects_a_changed_chunk_offset(stream):
    a, chunk, sub, r = stream
    off = r["chunk_off"].copy()
    off[17] += np.uint64(1)
    with pytest.raises(AssertionError):
        _check(a, chunk, sub, r, off=off)


def test_rejects_a_changed_piece_start(stream):
    a, chunk, sub, r = stream
    off = r["chunk_off"].copy()
    off[16:] += np.uint64(32)  # a whole later part moved by one word: pieces no longer add up
    w = np.concatenate([r["words"], np.zeros(1, np.uint32)])
    with pytest.raises(AssertionError):
        _check(a, chunk, sub, r, words=w, off=off)


def test_rejects_a_changed_sub_index(stream):
    a, chunk, sub, r = stream
    s = r["sub_lo"].copy()
    s[5000] += np.uint32(2)
    with pytest.raises(AssertionError):
        _check(a, chunk, sub, r, sub_lo=s)


def test_bits_equal_shifts():
    """bits_equal against a bit-by-bit comparison at every shift."""
    rng = np.random.default_rng(2)
    w = rng.integers(0, 1 << 32, size=9, dtype=np.uint64).astype(np.uint32)
    t = 9 * 32 - 5
    w[-1] &= np.uint32((0xFFFFFFFF << 5) & 0xFFFFFFFF)
    bits = np.unpackbits(w.astype(">u4").view(np.uint8))[:t]
    for s in range(32):
        allb = np.concatenate([rng.integers(0, 2, size=64 + s), bits, np.zeros(32, np.int64)]).astype(np.uint8)
        pad = (-allb.size) % 32
        allb = np.concatenate([allb, np.zeros(pad, np.uint8)])
        g = np.packbits(allb).view(">u4").astype(np.uint32)
        assert oracle_pieces.bits_equal(g, 64 + s, w, t, last=True)
        g2 = g.copy()
        k = 64 + s + t - 1  # the last bit of the range
        g2[k // 32] ^= np.uint32(1 << (31 - k % 32))
        assert not oracle_pieces.bits_equal(g2, 64 + s, w, t, last=False)
