"""GPU parity of the staged decoder's less common paths, each against the
CPU oracle bit for bit: codes longer than the peek table, waves whose
stream needs more than 8 bits per byte (staged in parts), the short last
wave of a stream, and corrupted sub-block indexes."""
import sys

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STAGED = [32, 64, 128, 256]
LUT_BITS = 10


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2306_11070_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def codec(P):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = P.Codec(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _starts(r, n, chunk, sub):
    """Absolute start bit of every sub-block, and the stream's end bit."""
    off = r["chunk_off"].astype(np.uint64)
    lo = r["sub_lo"].astype(np.uint64)
    j = np.arange(lo.size, dtype=np.uint64)
    base = off[(j * np.uint64(sub)) // np.uint64(chunk)]
    st = base + ((lo - (base & np.uint64(0xFFFFFFFF))) & np.uint64(0xFFFFFFFF))
    return np.append(st, off[-1])


def _max_wave_bits_per_byte(r, n, chunk, sub):
    st = _starts(r, n, chunk, sub)
    nitems = st.size - 1
    worst = 0.0
    for w0 in range(0, nitems, 64):
        w1 = min(w0 + 64, nitems)
        nbytes = min(w1 * sub, n) - w0 * sub
        worst = max(worst, float(st[w1] - st[w0]) / nbytes)
    return worst


def _skewed_tail(long_codes: bool, seed=0):
    """A run of one byte value, then a tail whose bytes need about 9 bits
    each; with long_codes a few values occur once, which gives them codes
    far longer than the peek table."""
    rng = np.random.default_rng(seed)
    head = np.zeros(200_000, np.uint8)
    if long_codes:
        tail = rng.integers(1, 250, size=40_000, dtype=np.uint8)
        tail[rng.choice(tail.size, 6, replace=False)] = np.arange(250, 256, dtype=np.uint8)
    else:
        tail = rng.integers(1, 256, size=40_000, dtype=np.uint8)
    return np.concatenate([head, tail, rng.integers(0, 1, size=1_234, dtype=np.uint8)])


def _roundtrip(codec, a, chunk, sub):
    st = codec.new_status()
    c = codec.compress(dev(a), chunk, sub, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    r = oracle.compress(a, chunk, sub=sub)
    nw = r["words"].size
    assert np.array_equal(c["words"].cpu().numpy().view(np.uint32)[:nw], r["words"])
    assert np.array_equal(c["chunk_off"].cpu().numpy().view(np.uint64), r["chunk_off"])
    out = codec.decompress(c, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(out.cpu().numpy(), a)
    return c, r


@pytest.mark.parametrize("sub", STAGED)
def test_staged_long_codes(codec, sub):
    """Zipf(1.3) over 256 values: codes past the 10-bit table, whole and short waves."""
    _say(f"staged long codes sub={sub}")
    a = datagen.zipf_iid(300_001, 21, 1.3, datagen.A256)
    r = oracle.compress(a, 4096, sub=sub)
    assert int(oracle.code_lengths(r["hist"]).max()) > LUT_BITS
    _roundtrip(codec, a, 4096, sub)


def _dyadic(L, seed):
    """About 1 MiB whose Huffman code has the lengths 1, 2, ..., L, L exactly
    (counts M * 2^(L-1), ..., M * 2, M, M, each count of a value halving the
    one before, shuffled): a code of L bits at most, with every length."""
    M = (1 << 20) >> L
    counts = [M << (L - 1 - i) for i in range(L)] + [M]
    a = np.repeat((np.arange(L + 1) * 7 + 3).astype(np.uint8), counts)
    np.random.default_rng(seed).shuffle(a)
    return a


@pytest.mark.parametrize("L", [11, 12, 13, 16])
@pytest.mark.parametrize("sub", [32, 64])
def test_staged_wide_table(codec, sub, L):
    """Codes just past the 10-bit table: the longer-code launch peeks 12 bits,
    so 11- and 12-bit codes decode from its table (two or three codes per
    window), 13 bits and more from its second table."""
    _say(f"staged wide table sub={sub} L={L}")
    a = _dyadic(L, seed=L)
    r = oracle.compress(a, 4096, sub=sub)
    assert int(oracle.code_lengths(r["hist"]).max()) == L
    _roundtrip(codec, a, 4096, sub)


WIDE_BITS, L2_MAX = 12, 2048  # the longer-code launch's peek bits and second-table capacity


def _second_table_entries(lengths):
    """Entries of the second table of a code (codes longer than WIDE_BITS bits):
    the WIDE_BITS-bit prefixes that the longer codes take, times 2^(maxLen - WIDE_BITS)."""
    ln = np.asarray(lengths)
    L = int(ln.max())
    if L <= WIDE_BITS:
        return 0
    cnt = np.bincount(ln[ln > 0], minlength=64)
    covered = sum(int(cnt[l]) << (WIDE_BITS - l) for l in range(1, WIDE_BITS + 1))
    return ((1 << WIDE_BITS) - covered) << (L - WIDE_BITS)


@pytest.mark.parametrize("s,max_len,table", [(1.6, 14, True), (1.8, 15, True), (2.0, 17, True), (2.2, 20, False)])
@pytest.mark.parametrize("sub", [32, 64])
def test_staged_second_table(codec, sub, s, max_len, table):
    """Codes past the 12-bit peek table: from the second table, two codes per
    window up to 16 bits and one past that, or by canonical search when the
    second table would pass its capacity; a ragged tail ends the stream."""
    _say(f"staged second table sub={sub} s={s}")
    a = datagen.zipf_iid((1 << 20) + 17, 3, s, datagen.A256)
    r = oracle.compress(a, 4096, sub=sub)
    ln = oracle.code_lengths(r["hist"])
    assert int(ln.max()) == max_len
    assert (0 < _second_table_entries(ln) <= L2_MAX) == table
    _roundtrip(codec, a, 4096, sub)


@pytest.mark.parametrize("long_codes", [False, True])
@pytest.mark.parametrize("sub", STAGED)
def test_staged_in_parts(codec, sub, long_codes):
    """Waves whose stream takes more than 8 bits per byte are staged in parts."""
    _say(f"staged in parts sub={sub} long={long_codes}")
    a = _skewed_tail(long_codes, seed=sub)
    chunk = 8192
    r = oracle.compress(a, chunk, sub=sub)
    ml = int(oracle.code_lengths(r["hist"]).max())
    assert (ml > LUT_BITS) == long_codes
    assert _max_wave_bits_per_byte(r, a.size, chunk, sub) > 8.05
    _roundtrip(codec, a, chunk, sub)


@pytest.mark.parametrize("n", [64 * 64 - 1, 64 * 64, 64 * 64 + 1, 3 * 64 * 64 + 17])
@pytest.mark.parametrize("sub", [32, 64])
def test_staged_short_last_wave(codec, sub, n):
    """Streams ending inside, at and just past a wave of whole sub-blocks."""
    _say(f"staged short last wave sub={sub} n={n}")
    _roundtrip(codec, datagen.markov(n, 31), 1024, sub)


@pytest.mark.parametrize("kind", ["markov", "zipf256_long"])
@pytest.mark.parametrize("sub", [32, 64, 128])
def test_staged_corrupt_index(codec, sub, kind):
    """A sub-block start moved by a few bits is reported, not decoded silently."""
    _say(f"staged corrupt index sub={sub} kind={kind}")
    a = datagen.markov(100_000, 32) if kind == "markov" else datagen.zipf_iid(100_000, 33, 1.6, datagen.A256)
    st = codec.new_status()
    c = codec.compress(dev(a), 1024, sub, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    bad = c["sub_lo"].clone()
    bad[70] += 3
    out = torch.empty(a.size, dtype=torch.uint8, device="cuda")
    codec.decode(c["words"], c["words"].numel(), c["chunk_off"], a.size, 1024, c["dcb"], sub_lo=bad,
                 sub_size=sub, out=out, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == -3
