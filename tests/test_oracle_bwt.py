"""Pins of the Method 3 oracle (block transform + move-to-front, CPU only):
worked examples from the literature (tests/golden/bwt_examples.txt),
brute-force sorted rotations on small blocks, inverse round trips, the
transform's invariants, and what the Huffman code gains from it."""
import os

import numpy as np
import pytest

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bwt_examples.txt")


def _golden(kind):
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, inp, exp, _ = [f.strip() for f in line.split("|")]
        if k == kind:
            out.append((inp, exp))
    assert out
    return out


@pytest.mark.parametrize("inp,exp", _golden("bwt"))
def test_bwt_worked_examples(inp, exp):
    last_s, row = exp.split()
    last, rows = oracle.bwt(inp.encode(), 64, 1)
    assert bytes(last) == last_s.encode()
    assert int(rows[0]) == int(row)
    assert bytes(oracle.unbwt(last, 64, 1, rows)) == inp.encode()


@pytest.mark.parametrize("inp,exp", _golden("mtf"))
def test_mtf_worked_example(inp, exp):
    got = oracle.mtf(inp.encode(), 1 << 20)
    assert got.tolist() == [int(v) for v in exp.split()]
    assert bytes(oracle.unmtf(got, 1 << 20)) == inp.encode()


def _brute_bwt(block: bytes):
    """Sorted cyclic rotations, written out (ties by start position)."""
    m = len(block)
    rots = sorted((block[i:] + block[:i], i) for i in range(m))
    last = bytes(r[-1] for r, _ in rots)
    row_of = {i: k for k, (_, i) in enumerate(rots)}
    return last, row_of


@pytest.mark.parametrize("seed", range(12))
def test_bwt_matches_brute_force_sorted_rotations(seed):
    rng = np.random.default_rng(seed)
    block, every = [16, 32, 64, 128][seed % 4], [1, 4, 16][seed % 3]
    n = int(rng.integers(1, 5 * block))
    alpha = [2, 3, 5, 256][seed % 4]
    a = rng.integers(0, alpha, size=n, dtype=np.uint16).astype(np.uint8)
    if seed % 5 == 0:
        a[: min(n, block)] = 7  # a constant block: every rotation equal, order by start
    last, rows = oracle.bwt(a, block, every)
    for lo in range(0, n, block):
        blk = bytes(a[lo:lo + block])
        bl, row_of = _brute_bwt(blk)
        assert bytes(last[lo:lo + len(blk)]) == bl
        for j in range(0, len(blk), every):
            assert int(rows[(lo + j) // every]) == row_of[j]
    assert np.array_equal(oracle.unbwt(last, block, every, rows), a)


@pytest.mark.parametrize("period", [1, 2, 3, 7])
def test_periodic_blocks_round_trip(period):
    """Equal rotations (a periodic block) still invert from the primary row."""
    unit = np.arange(period, dtype=np.uint8) * 37
    a = np.tile(unit, 3000)[: 4096 + 100]
    last, rows = oracle.bwt(a, 1024, 256)
    assert np.array_equal(oracle.unbwt(last, 1024, 256, rows), a)


def test_bwt_is_a_per_block_permutation_and_keeps_huffman_bits():
    """Each block's last column is a permutation of the block, so a byte
    Huffman code of it costs exactly the bits of the input (what makes the
    move-to-front step necessary for any gain)."""
    a = datagen.markov(300_000, 5)
    last, rows = oracle.bwt(a, 16384, 256)
    for lo in range(0, a.size, 16384):
        assert np.array_equal(np.sort(last[lo:lo + 16384]), np.sort(a[lo:lo + 16384]))
    h1, h2 = oracle.histogram(a), oracle.histogram(last)
    assert np.array_equal(h1, h2)
    assert oracle.total_bits(h2, oracle.code_lengths(h2)) == oracle.total_bits(h1, oracle.code_lengths(h1))


def test_mtf_runs_and_resets():
    a = np.array([5] * 10 + [9] * 3 + [5] * 2, dtype=np.uint8)
    assert oracle.mtf(a, 1024).tolist() == [5] + [0] * 9 + [9, 0, 0, 1, 0]
    # the list restarts at every block: the same block codes the same way
    b = np.concatenate([a, a])
    got = oracle.mtf(b, a.size)
    assert np.array_equal(got[: a.size], got[a.size:])
    rng = np.random.default_rng(0)
    c = rng.integers(0, 256, size=50_000, dtype=np.uint16).astype(np.uint8)
    assert np.array_equal(oracle.unmtf(oracle.mtf(c, 4096), 4096), c)


def test_method3_round_trip_and_gain_on_word_text():
    """Block transform + move-to-front + Huffman decodes back exactly, and on
    word-level text it codes in fewer bits than the Huffman code alone."""
    a = datagen.words(400_000, 9)
    r = oracle.compress_bwt(a, 16384, 256, 65536)
    m = oracle.decode(r["words"], r["chunk_off"], a.size, 65536, r["len"])
    assert np.array_equal(m, r["mtf"])
    assert np.array_equal(oracle.unbwt(oracle.unmtf(m, 16384), 16384, 256, r["rows"]), a)
    plain = oracle.compress(a, 65536)
    assert r["total_bits"] < 0.85 * plain["total_bits"]
