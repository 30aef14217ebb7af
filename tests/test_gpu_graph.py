"""The single-stream path captured in HIP graphs: huff_compress and
huff_decode queued on a stream that torch captures replay correctly, every
replay checked against the oracle, with eager library work, host
synchronisation and new input contents between the replays."""
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


@pytest.mark.parametrize("n,chunk,sub", [(3 * (1 << 20) + 77, 65536, 64), (200_001, 16384, 128), (9 * (16 << 20) + 5, 1 << 20, 128)])
def test_compress_decode_graph_replays(n, chunk, sub):
    import paper_2306_11070_amd as P
    P.load()
    _say(f"graph replays n={n} chunk={chunk} sub={sub}")
    codec = P.Codec(0)
    dev = "cuda"
    x = torch.empty(n, dtype=torch.uint8, device=dev)
    bufs = dict(hist=torch.empty(256, dtype=torch.int64, device=dev),
                dcb=torch.empty(P.DCB_BYTES, dtype=torch.uint8, device=dev),
                words=torch.empty((n + 3) // 4 + 4, dtype=torch.int32, device=dev),
                chunk_off=torch.empty((n + chunk - 1) // chunk + 1, dtype=torch.int64, device=dev),
                sub_lo=torch.empty((n + sub - 1) // sub + 1, dtype=torch.int32, device=dev))
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    x.copy_(torch.from_numpy(datagen.markov(n, 90)))
    codec.compress(x, chunk, sub, status=st, out=bufs)  # eager first call: sizes the context's workspaces
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    gc, gd = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(gc, stream=s):
            codec.compress(x, chunk, sub, status=st, out=bufs)
        with torch.cuda.graph(gd, stream=s):
            codec.decode(bufs["words"], bufs["words"].numel(), bufs["chunk_off"], n, chunk, bufs["dcb"],
                         bufs["sub_lo"], sub, out=out, status=st)
    torch.cuda.synchronize()
    for rep in range(4):
        a = datagen.markov(n, 91 + rep) if rep % 2 else datagen.zipf_iid(n, 95 + rep, 0.8, datagen.A256)
        x.copy_(torch.from_numpy(a))
        bufs["words"].fill_(-1)
        out.fill_(0)
        gc.replay()
        gd.replay()
        torch.cuda.synchronize()
        assert int(st.item()) == 0, rep
        r = oracle.compress(a, chunk, sub=sub)
        nw = r["words"].size
        assert np.array_equal(bufs["words"][:nw].cpu().numpy().view(np.uint32), r["words"]), rep
        assert np.array_equal(bufs["chunk_off"].cpu().numpy().view(np.uint64), r["chunk_off"]), rep
        assert np.array_equal(bufs["sub_lo"].cpu().numpy().view(np.uint32), r["sub_lo"]), rep
        assert torch.equal(out, x), rep
        # eager library work between replays
        c = codec.compress(x[: n // 2], chunk, sub)
        torch.cuda.synchronize()
        assert torch.equal(codec.decompress(c), x[: n // 2])
    codec.close()
