"""GPU test of huff_compress_noalloc (the compress entry point whose
workspaces live in the library's fixed device array): through the C ABI its
outputs equal huff_compress's on the same inputs, bit for bit (histogram,
codebook, words, chunk and sub-block offsets), on calls in a row whose inputs
shrink, and inputs past HUFF_NOALLOC_MAX_N are refused."""
import sys

import numpy as np
import pytest

import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _bufs(n, chunk, sub, P):
    dev = "cuda"
    return dict(hist=torch.empty(256, dtype=torch.int64, device=dev),
                dcb=torch.empty(P.DCB_BYTES, dtype=torch.uint8, device=dev),
                words=torch.full(((n + 3) // 4 + 4,), -1, dtype=torch.int32, device=dev),
                chunk_off=torch.full(((n + chunk - 1) // chunk + 1,), -1, dtype=torch.int64, device=dev),
                sub_lo=torch.full(((n + sub - 1) // sub + 1,), -1, dtype=torch.int32, device=dev) if sub else None)


def _same(c1, c2, sub):
    T = int(c2["chunk_off"][-1].item())
    nw = (T + 31) // 32
    assert torch.equal(c1["hist"], c2["hist"])
    assert torch.equal(c1["dcb"], c2["dcb"])
    assert torch.equal(c1["words"][:nw], c2["words"][:nw])
    assert torch.equal(c1["chunk_off"], c2["chunk_off"])
    if sub:
        assert torch.equal(c1["sub_lo"], c2["sub_lo"])


def test_noalloc_equals_compress_on_calls_in_a_row():
    import paper_2306_11070_amd as P
    P.load()
    codec = P.Codec(0)
    # the largest input first, then smaller ones: what a call leaves in the
    # shared workspace must not leak into the next
    cases = [("markov", P._abi.HUFF_NOALLOC_MAX_N, 1 << 20, 128),
             ("zipf", 3 * (16 << 20) + 12_345, 256 << 10, 64),
             ("markov", 100_003, 4096, 256),
             ("zipf", 17, 1024, 16)]
    for i, (kind, n, chunk, sub) in enumerate(cases):
        _say(f"noalloc call {i}: {kind} n={n} chunk={chunk} sub={sub}")
        a = datagen.markov(n, 70 + i) if kind == "markov" else datagen.zipf_iid(n, 80 + i, 0.8, datagen.A256)
        x = torch.from_numpy(a).cuda()
        st1, st2 = codec.new_status(), codec.new_status()
        c1 = codec.compress_noalloc(x, chunk, sub, out=_bufs(n, chunk, sub, P), status=st1)
        c2 = codec.compress(x, chunk, sub, status=st2, out=_bufs(n, chunk, sub, P))
        torch.cuda.synchronize()
        assert int(st1.item()) == 0 and int(st2.item()) == 0
        _same(c1, c2, sub)
        out = codec.decompress(c1, status=st1)
        torch.cuda.synchronize()
        assert int(st1.item()) == 0 and torch.equal(out, x)
        del x, c1, c2, out
    torch.cuda.empty_cache()
    codec.close()


def test_noalloc_refuses_inputs_past_its_workspace():
    import paper_2306_11070_amd as P
    P.load()
    codec = P.Codec(0)
    n = P._abi.HUFF_NOALLOC_MAX_N + 1
    x = torch.zeros(n, dtype=torch.uint8, device="cuda")
    _say("noalloc refuses n = max + 1")
    with pytest.raises(P.HuffError) as e:
        codec.compress_noalloc(x, 1 << 20, 0, out=_bufs(n, 1 << 20, 0, P))
    assert e.value.code == P._abi.HUFF_E_INVAL
    del x
    torch.cuda.empty_cache()
    codec.close()
