"""GPU parity of Method 3's block transform (huff_bwt, huff_mtf and their
inverses, through the C ABI) against the CPU oracle, bit for bit: the last
columns, the recorded rows, the move-to-front positions, the inverses, and
the whole Method 3 stream (transform + move-to-front + Huffman code)."""
import sys

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def codec():
    import paper_2306_11070_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = P.Codec(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _data(kind, n, seed=0):
    rng = np.random.default_rng(seed)
    if kind == "markov":
        return datagen.markov(n, 20 + seed)
    if kind == "words":
        return datagen.words(n, 30 + seed)
    if kind == "zipf256":
        return datagen.zipf_iid(n, 40 + seed, 0.8, datagen.A256)
    if kind == "uniform":
        return rng.integers(0, 256, size=n, dtype=np.uint16).astype(np.uint8)
    if kind == "const":
        return np.full(n, 0x61, dtype=np.uint8)
    if kind == "periodic":
        return np.tile(np.frombuffer(b"abcab", np.uint8), n // 5 + 1)[:n].copy()
    if kind == "two":
        return rng.choice(np.array([1, 200], np.uint8), size=n, p=[0.95, 0.05])
    raise KeyError(kind)


CASES = [
    ("markov", 1, 1024, 16), ("markov", 5, 1024, 16), ("words", 1023, 1024, 256), ("words", 1024, 1024, 1024),
    ("words", 1025, 1024, 64), ("markov", 16384, 16384, 256), ("words", 16385, 16384, 256),
    ("zipf256", 100_003, 16384, 128), ("uniform", 70_000, 4096, 16), ("const", 40_000, 16384, 256),
    ("periodic", 50_001, 8192, 512), ("two", 33_333, 2048, 32), ("words", 300_000, 16384, 16384),
    ("markov", 2 * 16384 + 3000, 16384, 4096),
]


@pytest.mark.parametrize("kind,n,block,every", CASES)
def test_bwt_mtf_and_inverses_match_oracle(codec, kind, n, block, every):
    _say(f"bwt kind={kind} n={n} block={block} every={every}")
    a = _data(kind, n, seed=n % 7)
    x = dev(a)
    last, rows = codec.bwt(x, block, every)
    ol, orows = oracle.bwt(a, block, every)
    torch.cuda.synchronize()
    assert np.array_equal(last.cpu().numpy(), ol)
    assert np.array_equal(rows.cpu().numpy().view(np.uint16)[: orows.size].astype(np.uint32), orows)
    m = codec.mtf(last, block)
    om = oracle.mtf(ol, block)
    torch.cuda.synchronize()
    assert np.array_equal(m.cpu().numpy(), om)
    back = codec.unmtf(m, block)
    st = codec.new_status()
    out = codec.unbwt(back, block, every, rows, status=st)
    torch.cuda.synchronize()
    assert np.array_equal(back.cpu().numpy(), ol)
    assert int(st.item()) == 0 and torch.equal(out, x)


def test_unbwt_of_oracle_transform(codec):
    """The inverse runs on the oracle's own transform (rows as u16)."""
    _say("unbwt of the oracle's transform")
    a = _data("words", 200_000, 3)
    ol, orows = oracle.bwt(a, 16384, 128)
    st = codec.new_status()
    out = codec.unbwt(dev(ol), 16384, 128, dev(orows.astype(np.uint16).view(np.int16)), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and np.array_equal(out.cpu().numpy(), a)


def test_unbwt_reports_bad_rows(codec):
    _say("unbwt bad rows")
    a = _data("markov", 5000, 1)
    last, rows = codec.bwt(dev(a), 4096, 256)
    bad = rows.clone()
    bad[-1] = 5000  # past the last block's 904 rows
    st = codec.new_status()
    codec.unbwt(last, 4096, 256, bad, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == -3


@pytest.mark.parametrize("kind,n", [("words", 3 * (1 << 20) + 77), ("markov", 1 << 20)])
def test_method3_stream_matches_oracle(codec, kind, n):
    """Transform + move-to-front + Huffman code: every word and index entry
    equals the oracle's Method 3 stream, and it decodes back exactly."""
    _say(f"method 3 stream kind={kind} n={n}")
    a = _data(kind, n, 5)
    x = dev(a)
    block, every, chunk, sub = 16384, 256, 256 << 10, 128
    st = codec.new_status()
    c = codec.compress_bwt(x, block, every, chunk, sub, status=st)
    r = oracle.compress_bwt(a, block, every, chunk, sub)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    nw = r["words"].size
    assert np.array_equal(c["words"].cpu().numpy().view(np.uint32)[:nw], r["words"])
    assert np.array_equal(c["chunk_off"].cpu().numpy().view(np.uint64), r["chunk_off"])
    assert np.array_equal(c["sub_lo"].cpu().numpy().view(np.uint32), r["sub_lo"])
    assert np.array_equal(c["rows"].cpu().numpy().view(np.uint16).astype(np.uint32), r["rows"])
    out = codec.decompress_bwt(c, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and torch.equal(out, x)
