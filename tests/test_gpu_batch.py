"""GPU parity of batches (huff_batch_*): every file of a batch is compared
with the CPU oracle on that file alone, bit for bit (histogram, code
lengths, words, segment index, decode index), decoded back, and compared
with the single-file calls.  Graph replays are checked on every replay."""
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


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host_u32(t, n=None):
    a = t.detach().cpu().numpy().view(np.uint32)
    return a if n is None else a[:n]


def host_u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


# sizes around tile (16 KiB) and scan-block edges, empty and one-byte files
SIZES = [0, 1, 17, 1000, 16383, 16384, 16385, 40_000, 100_003, 333_333, 0, 65_536, 5, 250_001]


def _file_data(i, n):
    kind = i % 5
    if kind == 0:
        return datagen.zipf_iid(n, 100 + i, 1.1)
    if kind == 1:
        return datagen.markov(n, 200 + i)
    if kind == 2:
        return datagen.zipf_iid(n, 300 + i, 0.8, datagen.A256)
    if kind == 3:
        return np.full(n, 0x41 + i, dtype=np.uint8)  # one distinct byte
    return np.random.default_rng(i).choice(np.array([7, 9, 200], np.uint8), size=n, p=[0.7, 0.2, 0.1])


def _check_file(f, a, chunk, sub, r=None):
    r = r or oracle.compress(a, chunk, sub=sub if sub else None)
    assert int(f["status"].item()) == 0
    assert np.array_equal(host_u64(f["hist"]), r["hist"])
    nw = r["words"].size
    assert np.array_equal(host_u32(f["words"], nw), r["words"])
    assert np.array_equal(host_u64(f["chunk_off"]), r["chunk_off"])
    if sub:
        assert np.array_equal(host_u32(f["sub_lo"]), r["sub_lo"])
    return r


@pytest.mark.parametrize("chunk,sub", [(4096, 64), (1024, 0), (65536, 256), (4096, 16)])
def test_batch_compress_decode_matches_oracle(P, codec, chunk, sub):
    _say(f"batch compress/decode chunk={chunk} sub={sub}")
    data = [_file_data(i, n) for i, n in enumerate(SIZES)]
    files = P.batch_buffers(codec, [dev(a) for a in data], chunk, sub)
    b = P.Batch(codec, files, chunk, sub)
    b.compress()
    torch.cuda.synchronize()
    for f, a in zip(files, data):
        _check_file(f, a, chunk, sub)
    b.decode()
    torch.cuda.synchronize()
    for f, a in zip(files, data):
        assert int(f["status"].item()) == 0
        assert np.array_equal(f["out"].cpu().numpy(), a)
    b.close()


def test_batch_equals_single_calls(P, codec):
    _say("batch vs single calls")
    chunk, sub = 2048, 128
    data = [_file_data(i, n) for i, n in enumerate([70_000, 16_384 * 3 + 7, 999, 123_457])]
    xs = [dev(a) for a in data]
    files = P.batch_buffers(codec, xs, chunk, sub)
    b = P.Batch(codec, files, chunk, sub)
    b.compress()
    for f, x in zip(files, xs):
        c = codec.compress(x, chunk, sub)
        torch.cuda.synchronize()
        nw = (int(host_u64(c["chunk_off"])[-1]) + 31) // 32
        assert torch.equal(c["dcb"], f["cb"])
        assert np.array_equal(host_u32(c["words"], nw), host_u32(f["words"], nw))
        assert torch.equal(c["chunk_off"], f["chunk_off"]) and torch.equal(c["sub_lo"], f["sub_lo"])
    b.close()


def test_batch_graph_replays(P, codec):
    """A captured batch replays correctly many times, with eager work and
    synchronisation between the replays, and after its inputs change."""
    _say("batch graph replays")
    chunk, sub = 4096, 64
    sizes = [30_000, 16_384, 1, 90_001, 0, 50_000]
    data = [_file_data(i + 7, n) for i, n in enumerate(sizes)]
    xs = [dev(a) for a in data]
    files = P.batch_buffers(codec, xs, chunk, sub)
    b = P.Batch(codec, files, chunk, sub)
    for rep in range(4):
        for f in files:
            f["words"].fill_(-1)
            f["chunk_off"].fill_(-1)
            f["out"].fill_(0)
        b.compress(graph=True)
        b.decode(graph=True)
        torch.cuda.synchronize()
        for f, a in zip(files, data):
            _check_file(f, a, chunk, sub)
            assert np.array_equal(f["out"].cpu().numpy(), a), rep
        # eager work between replays, then new contents in the same buffers
        codec.compress(xs[0], chunk, sub)
        torch.cuda.synchronize()
        for i, x in enumerate(xs):
            if x.numel():
                data[i] = _file_data(i + 50 + rep, x.numel())
                x.copy_(torch.from_numpy(data[i]))
    b.close()


def test_batch_encode_with_given_codebooks(P, codec):
    """HUFF_OP_ENCODE uses the codebooks already in the files (here uploaded
    from oracle lengths of other data, so not the file's own)."""
    _say("batch encode with given codebooks")
    chunk, sub = 4096, 0
    data = [_file_data(i, n) for i, n in enumerate([20_000, 70_000, 3])]
    xs = [dev(a) for a in data]
    files = P.batch_buffers(codec, xs, chunk, sub)
    hist_all = oracle.histogram(np.concatenate(data))
    ln = oracle.code_lengths(hist_all)
    cd = oracle.canonical_codes(ln)
    cbh = P.build_codebook(hist_all)
    for f in files:
        codec.codebook_upload(cbh, out=f["cb"])
    b = P.Batch(codec, files, chunk, sub)
    b.encode()
    torch.cuda.synchronize()
    for f, a in zip(files, data):
        w, off = oracle.encode(a, ln, cd, chunk)
        assert int(f["status"].item()) == 0
        assert np.array_equal(host_u32(f["words"], w.size), w)
        assert np.array_equal(host_u64(f["chunk_off"]), off)
    b.close()


def test_batch_unaligned_inputs(P, codec):
    _say("batch unaligned inputs")
    chunk, sub = 1024, 32
    data = [_file_data(i, n) for i, n in enumerate([50_000, 16_385, 777])]
    xs = []
    for i, a in enumerate(data):
        off = 3 + 4 * i
        xs.append(dev(np.concatenate([np.zeros(off, np.uint8), a]))[off:])
    files = P.batch_buffers(codec, xs, chunk, sub)
    b = P.Batch(codec, files, chunk, sub)
    b.compress()
    b.decode()
    torch.cuda.synchronize()
    for f, a in zip(files, data):
        _check_file(f, a, chunk, sub)
        assert np.array_equal(f["out"].cpu().numpy(), a)
    b.close()


def test_batch_many_files_log_uniform(P, codec):
    """A small sample of the many-file workload (log-uniform sizes, per-file
    Zipf exponent and alphabet), checked file by file."""
    _say("batch many files")
    chunk, sub = 65536, 256
    data = [datagen.batch_file(5, i, size_lo=4096, size_hi=1 << 18) for i in range(96)]
    files = P.batch_buffers(codec, [dev(a) for a in data], chunk, sub)
    b = P.Batch(codec, files, chunk, sub)
    b.compress(graph=True)
    b.decode(graph=True)
    torch.cuda.synchronize()
    for f, a in zip(files, data):
        _check_file(f, a, chunk, sub)
        assert np.array_equal(f["out"].cpu().numpy(), a)
    b.close()


def test_batch_decode_needs_outputs(P, codec):
    """A plan whose non-empty file has no output buffer refuses to decode
    (before any launch) and still compresses."""
    _say("batch decode without outputs")
    data = [_file_data(i, n) for i, n in enumerate([5_000, 0, 20_000])]
    files = P.batch_buffers(codec, [dev(a) for a in data], 4096, 64, decode=False)
    b = P.Batch(codec, files, 4096, 64)
    with pytest.raises(P.HuffError):
        b.decode()
    b.compress()
    torch.cuda.synchronize()
    for f, a in zip(files, data):
        _check_file(f, a, 4096, 64)
    b.close()



def test_batch_scan_carries_across_blocks(P, codec):
    """Files that open and close across the 16 MiB scan blocks (1024 tiles of
    16 KiB): a file that starts exactly at a block's first tile, files that
    start inside a block and end in a later one, a file that covers a whole
    block, and empty and tiny files between them.  Every file is compared
    with the oracle on that file alone (histogram, words, chunk and
    sub-block offsets), and decoded back."""
    from concurrent.futures import ThreadPoolExecutor

    MiB = 1 << 20
    # tile starts: 0, 1024 (block 1's first tile), 2304, 2305, 2305, 3074,
    # 3074 (covers block 4), 5635, 5636; 6660 tiles in 7 blocks
    sizes = [16 * MiB, 20 * MiB, 1, 0, 12 * MiB + 5, 0, 40 * MiB + 7, 3, 16 * MiB - 16384 + 1]
    _say(f"batch across scan blocks: {len(sizes)} files, {sum(sizes)} bytes")
    data = [_file_data(i, n) for i, n in enumerate(sizes)]
    chunk, sub = 256 << 10, 128
    xs = [dev(a) for a in data]
    files = P.batch_buffers(codec, xs, chunk, sub)
    b = P.Batch(codec, files, chunk, sub)
    for rep in range(2):
        for f in files:
            f["words"].fill_(-1)
            f["chunk_off"].fill_(-1)
            f["sub_lo"].fill_(-1)
            f["out"].fill_(0)
        b.compress(graph=rep == 1)
        b.decode(graph=rep == 1)
        torch.cuda.synchronize()
        with ThreadPoolExecutor(8) as ex:
            refs = list(ex.map(lambda a: oracle.compress(a, chunk, sub=sub), data))
        for i, (f, a, r) in enumerate(zip(files, data, refs)):
            _check_file(f, a, chunk, sub, r)
            assert torch.equal(f["out"], xs[i]), (rep, i)
    b.close()


def test_batch_codes_past_the_table(P, codec):
    """Files whose longest codes are 9, 11, 12, 13 and 15 bits in one batch,
    and Zipf files with 14-, 17- and 20-bit codes: the longer-code decode
    launch takes the files past the 10-bit table, decodes codes of up to 12
    bits from its 12-bit table and longer ones from its second table, or by
    canonical search where that table would pass its capacity (the 20-bit
    file).  Every file against the oracle alone, and decoded back."""
    data = []
    for i, L in enumerate([9, 11, 12, 13, 15, 11]):
        M = (1 << 19) >> L
        counts = [M << (L - 1 - k) for k in range(L)] + [M]
        a = np.repeat((np.arange(L + 1) * 11 + 1).astype(np.uint8), counts)
        np.random.default_rng(40 + i).shuffle(a)
        data.append(a[: a.size - 3 * i])  # ragged ends
    for i, s in enumerate([1.6, 2.0, 2.2]):
        data.append(datagen.zipf_iid((1 << 20) + 5 * i, 3, s, datagen.A256))
    want = [9, 11, 12, 13, 15, 11, 14, 17, 20]
    assert [int(oracle.code_lengths(np.bincount(a, minlength=256)).max()) for a in data] == want
    _say(f"batch past the table: {len(data)} files")
    for sub in (32, 64):
        chunk = 16384
        xs = [dev(a) for a in data]
        files = P.batch_buffers(codec, xs, chunk, sub)
        b = P.Batch(codec, files, chunk, sub)
        b.compress()
        b.decode()
        torch.cuda.synchronize()
        for f, a, x in zip(files, data, xs):
            _check_file(f, a, chunk, sub)
            assert torch.equal(f["out"], x)
        b.close()


@pytest.mark.parametrize("kind", ["all_short", "all_long", "alternating"])
def test_batch_decode_block_modes(P, codec, kind):
    """The two staged decode launches split a batch's blocks by the per-block
    mode map: batches whose files all fit the peek table, all pass it, or
    alternate file by file (small and large files, so blocks of both modes
    sit side by side), decoded twice (the map is rewritten at every decode)."""
    sizes = [70_001, 3, 300_017, 16_384, 1 << 20, 65_536 + 9]
    data = []
    for i, n in enumerate(sizes):
        long_codes = kind == "all_long" or (kind == "alternating" and i % 2 == 1)
        s = 1.8 if long_codes else 1.0
        data.append(datagen.zipf_iid(n, 60 + i, s, datagen.A256, 256 if long_codes else 64))
    for i, a in enumerate(data):
        if a.size > 1000:  # the 3-byte file has a short code whatever its source
            ml = int(oracle.code_lengths(np.bincount(a, minlength=256)).max())
            assert (ml > 10) == (kind == "all_long" or (kind == "alternating" and i % 2 == 1)), (i, ml)
    _say(f"batch block modes {kind}")
    xs = [dev(a) for a in data]
    files = P.batch_buffers(codec, xs, 16384, 64)
    b = P.Batch(codec, files, 16384, 64)
    b.compress(graph=True)
    for rep in range(2):
        for f in files:
            f["out"].zero_()
        b.decode(graph=True)
        torch.cuda.synchronize()
        for f, a, x in zip(files, data, xs):
            _check_file(f, a, 16384, 64)
            assert torch.equal(f["out"], x), (kind, rep)
    b.close()
