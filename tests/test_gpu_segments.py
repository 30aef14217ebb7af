"""GPU parity of per-segment codebooks within one stream (Method 2 with a
tree per segment): every segment against the CPU oracle on that segment
alone, bit for bit, the decoded stream against the input, and the size
relation that holds for optimal codes: each segment coded with its own
Huffman code takes at most the bits the whole stream's code spends on it."""
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


def _u32(t, n):
    return t.detach().cpu().numpy().view(np.uint32)[:n]


@pytest.mark.parametrize("seg,chunk,sub,n", [(256 << 10, 64 << 10, 128, (3 << 20) + 12345),
                                             (16 << 10, 4096, 64, 100_003),
                                             (4096, 1024, 0, 4096 * 7)])
def test_segments_match_oracle_per_segment(P, codec, seg, chunk, sub, n):
    _say(f"segments seg={seg} chunk={chunk} sub={sub} n={n}")
    a = datagen.markov(n, 77)
    x = torch.from_numpy(a).cuda()
    sg = P.Segments(codec, x, seg, chunk, sub)
    sg.compress(graph=True)
    sg.decode(graph=True)
    torch.cuda.synchronize()
    bits = sg.segment_bits()
    for i, f in enumerate(sg.files):
        part = a[i * seg:(i + 1) * seg]
        r = oracle.compress(part, chunk, sub=sub if sub else None)
        assert int(f["status"].item()) == 0, i
        assert np.array_equal(f["hist"].cpu().numpy().view(np.uint64), r["hist"]), i
        assert np.array_equal(_u32(f["words"], r["words"].size), r["words"]), i
        assert np.array_equal(f["chunk_off"].cpu().numpy().view(np.uint64), r["chunk_off"]), i
        if sub:
            assert np.array_equal(f["sub_lo"].cpu().numpy().view(np.uint32), r["sub_lo"]), i
        assert bits[i] == int(r["chunk_off"][-1])
    assert torch.equal(sg.out, x)
    # a segment's own code is optimal for it: never longer than the global code on it
    ln = oracle.code_lengths(oracle.histogram(a))
    for i in range(sg.nseg):
        part = a[i * seg:(i + 1) * seg]
        assert bits[i] <= oracle.total_bits(oracle.histogram(part), ln), i
    sg.close()


def test_segments_reject_unaligned_size(P, codec):
    x = torch.zeros(1000, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        P.Segments(codec, x, 1000, 1024)
