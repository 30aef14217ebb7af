"""Host replay of the GPU path's addressing at n = 2^31 (CPU only, slow).

A run of the 2 GiB parity test once ended in a GPU memory fault (1 MiB
chunks, 4096-byte sub-blocks, an encode kernel that has since been taken
out).  This test recomputes, on the host, every global address, element
count and buffer range that the launches of a 2 GiB compress and decode
would use -- from the real per-tile and per-64-byte-unit code bits of both
2 GiB workloads -- and checks each against the allocation the Python binding
and the context make for it:

  * the launch shapes of api.cpp (histogram, tile bits, the segmented scan
    with its block carries, the encode grid (two tiles per workgroup), the direct decoder
    at 4096-byte sub-blocks and the staged decoder at 64 and 128);
  * k_hist's 16-byte loads and per-tile histogram rows; k_tile_bits_hist's
    rows; the scans' tile and block entries;
  * k_encode's clamped prefetch loads, the 32 bytes before each tile, the
    tile-offset and carry loads, the segment and decode index stores, and the
    word range each tile stores (and that it fits the LDS rows it is put
    together in);
  * the decoders' start and end bits, the direct reader's unguarded 16-byte
    loads and the staged decoder's staging ranges and output stores;
  * for the encode kernel that ran when the fault happened: the byte range
    of every buffer descriptor it built and the offsets of every store it
    issued (stores meant to write nothing used an offset of 2^31, which the
    descriptor's range check drops).

Every check passes: at n = 2^31 none of these accesses leaves its
allocation, so this replay does not show a cause for the fault (it is kept
as a record and a regression check of the addressing).
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.slow

N = 1 << 31
TILE = 16384          # encode / histogram tile (256 threads x 64 bytes)
UNIT = 64
SCAN = 1024           # tiles per scan block
CHUNK = 1 << 20
NUM_CUS = 256


def _bits(name):
    a = datagen.workload(name)
    assert a.size == N
    h = np.bincount(a, minlength=256).astype(np.uint64)
    ln = oracle.code_lengths(h)
    unit = np.empty(N // UNIT, dtype=np.uint32)
    step = 1 << 26  # bytes per slice, to bound the temporary
    for lo in range(0, N, step):
        unit[lo // UNIT:(lo + step) // UNIT] = ln[a[lo:lo + step]].reshape(-1, UNIT).sum(axis=1, dtype=np.uint32)
    del a
    b = np.zeros(unit.size + 1, dtype=np.uint64)  # stream bit of every unit, and T
    np.cumsum(unit, dtype=np.uint64, out=b[1:])
    return ln, unit, b


@pytest.fixture(scope="module", params=["markov_2GiB", "zipf256_2GiB"])
def stream(request):
    return (request.param,) + _bits(request.param)


def _alloc():
    """Element counts of what the binding and the context allocate for one
    2 GiB compress (torch.empty sizes in Codec.compress; ensure_tiles)."""
    ntiles = N // TILE
    return dict(words=(N + 3) // 4 + 4, chunk_off=N // CHUNK + 1, tile_cap=max(ntiles, 4096),
                blk=max(ntiles, 4096) // SCAN + 1)


def test_histogram_and_scan_addressing(stream):
    name, ln, unit, b = stream
    al = _alloc()
    ntiles = N // TILE
    # launch_hist_only: blocks = min(hist_blocks, ntiles), at least n >> 31 + 1
    blocks = max(min(NUM_CUS * 16, ntiles), (N >> 31) + 1)
    tpb = -(-ntiles // blocks)
    blocks = -(-ntiles // tpb)
    assert tpb * TILE < 1 << 31  # each workgroup counts fewer than 2^31 bytes (u32 LDS counters)
    t = np.arange(ntiles, dtype=np.uint64)
    q_last = t * TILE + TILE // 2 + 511 * 16  # the highest 16-byte load of each tile (thread 511)
    assert int(q_last.max()) + 16 <= N
    assert (ntiles - 1) * 256 + 255 < al["tile_cap"] * 256  # tile_hist row of the last tile
    assert blocks <= ntiles
    # k_tile_bits_hist: one wave per tile; u16 counts (<= 16384) and u32 bits
    tile_bits = unit.reshape(ntiles, TILE // UNIT).sum(axis=1, dtype=np.uint64)
    assert int(tile_bits.max()) < 1 << 32
    # scan: more than kInlineCarryBlocks blocks -> the segmented scan and k_blk_scan
    nblk = -(-ntiles // SCAN)
    assert nblk > 8 and nblk <= al["blk"]
    per_blk = tile_bits.reshape(nblk, SCAN).sum(axis=1)
    assert int(per_blk.max()) < 1 << 32  # tile_local is u32 within a block
    assert int(b[-1]) < 1 << 62  # block tails keep 62 bits


def test_encode_addressing(stream):
    name, ln, unit, b = stream
    al = _alloc()
    ntiles = N // TILE
    max_len = int(ln.max())
    grid = min(ntiles, NUM_CUS * 256)  # 65536 workgroups: two tiles each at 2 GiB
    tiles = np.arange(ntiles, dtype=np.uint64)
    # workgroup w takes tiles w, w + grid, ...; the next tile's loads are issued
    # only while that tile exists
    nxt = tiles + np.uint64(grid)
    assert int(nxt[nxt < ntiles].max()) < ntiles and -(-ntiles // grid) == 2
    # prefetch: four clamped 16-byte loads per thread, all whole blocks of the input
    q = tiles * TILE + 255 * UNIT + 48
    assert int(q.max()) + 16 <= N
    # the 32 bytes before a tile (lanes 0..7, tiles after the first)
    bo = tiles[1:] * TILE - 32 + 4 * 7
    assert int(bo.max()) + 4 <= N
    assert ntiles - 1 < al["tile_cap"] and (ntiles - 1) // SCAN < al["blk"]
    # words each tile stores: those whose last bit lies in the tile, plus the
    # stream's final partial word after the last tile
    S = b[:-1:TILE // UNIT]  # first stream bit of each tile
    E = np.append(S[1:], b[-1])
    T = int(b[-1])
    ws = S >> np.uint64(5)
    nwt = (E >> np.uint64(5)) - ws
    nwt[-1] += np.uint64(1 if T & 31 else 0)
    assert int(((E + np.uint64(31)) >> np.uint64(5)).max()) <= al["words"]  # every tile fits (capOK)
    assert int((ws + nwt).max()) <= al["words"]
    # the LDS rows a tile's words are put together in
    lin_words = (UNIT * 16 // 32 + 1 - (UNIT * 8 // 32 + 1)) * 257
    all_words = (UNIT * 16 // 32 + 1) * 257
    if max_len <= 8:
        assert int(nwt.max()) <= lin_words
    elif max_len <= 10:
        assert int(nwt.max()) <= all_words
    # segment and decode index stores
    for sub in (64, 128, 4096):
        nsub = N // sub
        assert (N - 1) // sub < nsub + 1 and N // sub <= nsub  # last unit start and the end entry
        assert int(((b[:-1] if sub == UNIT else b[:-1:sub // UNIT]) & np.uint64(0xFFFFFFFF)).size) == nsub
    assert (N - UNIT) // CHUNK < al["chunk_off"] and N // CHUNK < al["chunk_off"]
    # no chunk spans 2^32 bits (the decode index keeps low 32 bits)
    c = b[::CHUNK // UNIT]
    assert int(np.diff(c).max()) < 1 << 32


def test_direct_decoder_addressing_4096(stream):
    """The direct decoder at 4096-byte sub-blocks, the configuration of the
    run that faulted: start and end bits, the reader's unguarded loads."""
    name, ln, unit, b = stream
    al = _alloc()
    sub = 4096
    starts = b[:-1:sub // UNIT]
    ends = np.append(starts[1:], b[-1])
    nw = al["words"]  # the binding passes words.numel() as nwords
    assert np.all(starts <= ends) and int(ends.max()) <= nw * 32
    # BitReader: vectors from (start >> 5) >> 2; a refill never reads more than
    # one vector past the one holding the item's last bit, plus the one in flight
    first_vec = (starts >> np.uint64(5)) >> np.uint64(2)
    last_vec = ((ends + np.uint64(63)) >> np.uint64(5) >> np.uint64(2)) + np.uint64(2)
    unguarded = np.minimum(last_vec, np.uint64(nw // 4 - 1))  # vec[vi] only when (vi + 1) * 4 <= nwords
    assert int(((unguarded + np.uint64(1)) * np.uint64(4)).max()) <= nw
    assert int(first_vec.max()) < nw // 4 + 1
    # launch: 256-lane workgroups over 2^19 items; output 16-byte groups inside n
    nitems = N // sub
    blocks = -(-nitems // 256)
    assert blocks * 256 >= nitems and (nitems - 1) * sub + sub <= N


@pytest.mark.parametrize("sub", [64, 128])
def test_staged_decoder_addressing(stream, sub):
    name, ln, unit, b = stream
    al = _alloc()
    nw = al["words"]
    starts = b[:-1:sub // UNIT] if sub >= UNIT else None
    ends = np.append(starts[1:], b[-1])
    nitems = N // sub
    k_in_words = 64 * sub // 4 + 8
    # each wave: 64 items; staged words [base, base + cnt) with base a multiple of 4
    ws = starts[::64]
    we = ends[63::64]
    base = (ws >> np.uint64(5)) & ~np.uint64(3)
    cnt = ((we + np.uint64(31)) >> np.uint64(5)) - base
    staged = np.minimum((cnt + np.uint64(3)) >> np.uint64(2), np.uint64(k_in_words // 4)) * np.uint64(4)
    assert int((base + staged).max()) <= nw + 3  # reads past nwords are guarded word by word
    parts = cnt + np.uint64(4) > np.uint64(k_in_words)
    assert nitems % 64 == 0
    # every output store lies inside the n-byte output
    assert (nitems // 64 - 1) * 64 * sub + 64 * sub <= N
    if int(ln.max()) <= 8:
        assert not parts.any()  # at most 8 bits per byte: every wave fits its buffer


def test_faulted_variant_descriptors(stream):
    """The encode kernel that ran when the fault happened stored through
    buffer descriptors (range clamped to 2^31 - 1 bytes) and gave stores meant
    to write nothing the offset 2^31.  Every store it meant to make falls
    inside its descriptor's range and inside the allocation, and every store
    meant to write nothing falls outside the range (so it is dropped)."""
    name, ln, unit, b = stream
    al = _alloc()
    nw_cap = al["words"]
    ntiles = N // TILE
    S = b[:-1:TILE // UNIT]
    tw = S >> np.uint64(5)
    rng = np.minimum((np.uint64(nw_cap) - tw) * np.uint64(4), np.uint64(0x7FFFFFFF))
    # per thread: words [w0, e>>5 (+1 for the last)) at byte offsets (w - tw) * 4
    w0 = b[:-1] >> np.uint64(5)
    wend = b[1:] >> np.uint64(5)
    wend[-1] += np.uint64(1 if int(b[-1]) & 31 else 0)
    tile_of = np.arange(w0.size, dtype=np.uint64) // np.uint64(TILE // UNIT)
    last_off = (np.maximum(wend, w0 + np.uint64(1)) - np.uint64(1) - tw[tile_of]) * np.uint64(4)
    assert np.all(last_off + np.uint64(4) <= rng[tile_of])  # every meant store is in range
    assert int((tw * np.uint64(4) + rng).max()) <= nw_cap * 4  # ranges stay inside the words allocation
    drop = np.uint64(0x80000000)
    assert np.all(drop >= rng)  # stores meant to write nothing are out of range
    # where a dropped store's address would be: inside the words allocation
    # only for the first tiles (base + 2^31 < words + 4 * nw_cap)
    inside = (tw * np.uint64(4) + drop) < np.uint64(nw_cap * 4)
    assert int(inside.sum()) <= 4 and bool(inside[0])
    # segment-index descriptors
    nch = N // CHUNK + 1
    c0 = (np.arange(ntiles, dtype=np.uint64) * np.uint64(TILE)) >> np.uint64(20)
    assert np.all((np.uint64(nch) - c0) * np.uint64(8) <= np.uint64(0x7FFFFFFF))
