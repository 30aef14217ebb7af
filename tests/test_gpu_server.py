"""GPU tests of the request server (huff_server_*): served results against
the CPU oracle, the same request alone and in a mix of concurrent requests
(bit-exact), admission against the memory budget, deferred release, and the
open-loop replay driver."""
import ctypes
import sys

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

OP_C, OP_D = 0, 2


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2306_11070_amd as P
    P.load()
    return P


_hip = None


def d2h(ptr: int, nbytes: int, dtype=np.uint8) -> np.ndarray:
    """Copies device memory at `ptr` to a host array (test helper)."""
    global _hip
    if _hip is None:
        torch.cuda.init()
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    out = np.empty(nbytes, dtype=np.uint8)
    if nbytes:
        assert _hip.hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0  # device to host
    return out.view(dtype)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _stream_host(srv, handle):
    i = srv.stream(handle)
    T = i["total_bits"]
    nw = (T + 31) // 32
    n = i["n"]
    nch = (n + srv.chunk_size - 1) // srv.chunk_size
    words = d2h(i["words"], nw * 4, np.uint32)
    off = d2h(i["chunk_off"], (nch + 1) * 8, np.uint64)
    sub = None
    if srv.sub_size:
        nsub = (n + srv.sub_size - 1) // srv.sub_size
        sub = d2h(i["sub_lo"], (nsub + 1) * 4, np.uint32)
    return words, off, sub


def _req_data(i, n):
    return datagen.markov(n, 1000 + i) if i % 3 else datagen.zipf_iid(n, 2000 + i, 1.1)


def test_server_results_match_oracle(P):
    _say("server vs oracle")
    srv = P.Server(mem_budget=256 << 20, chunk_size=16384, sub_size=64)
    sizes = [1, 1000, 16384, 16385, 100_003, 555_555, 0, 2_000_001]
    data = [_req_data(i, n) for i, n in enumerate(sizes)]
    xs = [dev(a) for a in data]
    tickets = [srv.submit_compress(x) for x in xs]
    res = [srv.wait(t) for t in tickets]
    dts = []
    for r, a in zip(res, data):
        assert r["status"] == 0
        words, off, sub = _stream_host(srv, r["handle"])
        ref = oracle.compress(a, 16384, sub=64)
        assert np.array_equal(words, ref["words"])
        assert np.array_equal(off, ref["chunk_off"])
        assert np.array_equal(sub, ref["sub_lo"])
        assert r["out_bytes"] == (int(ref["chunk_off"][-1]) + 7) // 8
        dts.append(srv.submit_decode(r["handle"]))
    for t, a in zip(dts, data):
        r = srv.wait(t)
        assert r["status"] == 0 and r["out_bytes"] == a.size
        assert np.array_equal(d2h(srv.stream(r["handle"])["out"], a.size), a)
        srv.release(r["handle"])
    for r in res:
        srv.release(r["handle"])
    st = srv.stats()
    assert st["mem_used"] == 0 and st["waiting"] == 0
    srv.close()


def test_server_alone_equals_mix(P):
    """Each request's result is the same served alone and served among many
    concurrent requests of mixed sizes and kinds."""
    _say("server alone vs mix")
    srv = P.Server(mem_budget=1 << 30, nslots=3, max_batch=64, chunk_size=65536, sub_size=128)
    rng = np.random.default_rng(7)
    probe = [_req_data(i, int(n)) for i, n in enumerate([300_000, 5_000, 1_234_567])]
    xp = [dev(a) for a in probe]
    alone = []
    for x in xp:
        r = srv.wait(srv.submit_compress(x))
        assert r["status"] == 0
        w, o, s = _stream_host(srv, r["handle"])
        d = srv.wait(srv.submit_decode(r["handle"]))
        alone.append((w, o, s, d2h(srv.stream(d["handle"])["out"], x.numel())))
        srv.release(d["handle"])
        srv.release(r["handle"])
    # the mix: background compress and decode requests around the probes
    bg = [_req_data(10 + i, int(rng.integers(1, 3_000_000))) for i in range(40)]
    xb = [dev(a) for a in bg]
    base = [srv.wait(srv.submit_compress(x)) for x in xb[:10]]
    tickets = []
    for i, x in enumerate(xb[10:]):
        tickets.append(("c", srv.submit_compress(x)))
        if i % 3 == 0:
            tickets.append(("d", srv.submit_decode(base[i % 10]["handle"])))
        if i in (5, 15, 25):
            k = (5, 15, 25).index(i)
            tickets.append(("p", k, srv.submit_compress(xp[k])))
    got = {}
    for t in tickets:
        r = srv.wait(t[-1])
        assert r["status"] == 0
        if t[0] == "p":
            got[t[1]] = r
        elif t[0] == "d":
            srv.release(r["handle"])
        else:
            srv.release(r["handle"])
    for k, r in got.items():
        w, o, s = _stream_host(srv, r["handle"])
        assert np.array_equal(w, alone[k][0]) and np.array_equal(o, alone[k][1]) and np.array_equal(s, alone[k][2])
        d = srv.wait(srv.submit_decode(r["handle"]))
        assert np.array_equal(d2h(srv.stream(d["handle"])["out"], probe[k].size), alone[k][3])
        assert np.array_equal(alone[k][3], probe[k])
        srv.release(d["handle"])
        srv.release(r["handle"])
    st = srv.stats()
    assert st["batches"] >= 2
    for b in base:
        srv.release(b["handle"])
    srv.close()


def test_server_admission_under_budget(P):
    """Requests that together exceed the budget are admitted as memory frees;
    one that can never fit is refused at submit."""
    _say("server admission")
    budget = 12 << 20
    srv = P.Server(mem_budget=budget, chunk_size=16384)
    with pytest.raises(P.HuffError):
        srv.submit_compress(dev(np.zeros(16 << 20, np.uint8)))
    data = [_req_data(i, 1_500_000) for i in range(12)]
    xs = [dev(a) for a in data]
    tickets = [srv.submit_compress(x) for x in xs]
    for t, a in zip(tickets, data):
        r = srv.wait(t)
        assert r["status"] == 0
        words, off, _ = _stream_host(srv, r["handle"])
        ref = oracle.compress(a, 16384)
        assert np.array_equal(words, ref["words"]) and np.array_equal(off, ref["chunk_off"])
        srv.release(r["handle"])  # frees room for the ones still waiting
    st = srv.stats()
    assert st["mem_peak"] <= budget and st["mem_used"] == 0
    srv.close()


def test_server_release_is_deferred_while_decoding(P):
    _say("server deferred release")
    srv = P.Server(mem_budget=64 << 20, chunk_size=16384, sub_size=256)
    a = _req_data(3, 3_000_000)
    r = srv.wait(srv.submit_compress(dev(a)))
    t = srv.submit_decode(r["handle"])
    srv.release(r["handle"])  # the queued decode still reads it
    d = srv.wait(t)
    assert d["status"] == 0
    assert np.array_equal(d2h(srv.stream(d["handle"])["out"], a.size), a)
    with pytest.raises(P.HuffError):
        srv.stream(r["handle"])
    srv.release(d["handle"])
    assert srv.stats()["mem_used"] == 0
    srv.close()


def test_server_replay_open_loop(P):
    _say("server replay")
    srv = P.Server(mem_budget=512 << 20, chunk_size=65536, sub_size=256)
    data = [_req_data(i, n) for i, n in enumerate([10_000, 700_000, 3_000_000, 64, 250_000])]
    xs = [dev(a) for a in data]
    pre = [srv.wait(srv.submit_compress(x)) for x in xs]
    reqs, arr = [], []
    rng = np.random.default_rng(3)
    t = 0.0
    for i in range(60):
        k = int(rng.integers(0, len(xs)))
        if rng.random() < 0.7:
            reqs.append((OP_C, xs[k], 0))
        else:
            reqs.append((OP_D, None, pre[k]["handle"]))
        t += float(rng.exponential(0.0005))
        arr.append(t)
    res = srv.replay(reqs, arr)
    for (op, x, h), r in zip(reqs, res):
        assert r["status"] == 0
        assert r["t_done"] >= r["t_start"] >= r["t_submit"] > 0
        if op == OP_C:
            k = next(i for i, y in enumerate(xs) if y is x)
            w, o, _ = _stream_host(srv, r["handle"])
            w0, o0, _ = _stream_host(srv, pre[k]["handle"])
            assert np.array_equal(w, w0) and np.array_equal(o, o0)
        srv.release(r["handle"])
    for p in pre:
        srv.release(p["handle"])
    assert srv.stats()["mem_used"] == 0
    srv.close()


def test_server_checks_results_against_oracle(P):
    """Requests that carry the oracle's result are compared with it on the
    device: equal results keep status 0; a changed word, a wrong length or a
    changed decoded byte gives HUFF_E_MISMATCH (-9).  Also through the
    open-loop replay with every result discarded after its check."""
    _say("server result checks")
    chunk, sub = 65536, 128
    srv = P.Server(mem_budget=512 << 20, nslots=2, chunk_size=chunk, sub_size=sub)
    data = [_req_data(i, n) for i, n in enumerate([1, 70_000, 1_000_003, 16_384, 2_500_000])]
    refs = [oracle.compress(a, chunk) for a in data]
    xs = [dev(a) for a in data]
    want = [dev(np.concatenate([r["words"], np.zeros(4, np.uint32)]).view(np.int32)) for r in refs]
    bits = [int(r["total_bits"]) for r in refs]
    res = [srv.wait(srv.submit_compress(x, expect=w, expect_bits=b)) for x, w, b in zip(xs, want, bits)]
    assert [r["status"] for r in res] == [0] * len(xs)
    # a changed word, then a wrong length
    bad = want[2].clone()
    bad[1234] ^= 1 << 7
    assert srv.wait(srv.submit_compress(xs[2], expect=bad, expect_bits=bits[2]))["status"] == -9
    assert srv.wait(srv.submit_compress(xs[2], expect=want[2], expect_bits=bits[2] + 1))["status"] == -9
    # decodes against the original bytes
    dec = [srv.wait(srv.submit_decode(r["handle"], expect=x)) for r, x in zip(res, xs)]
    assert [d["status"] for d in dec] == [0] * len(xs)
    for d in dec:
        srv.release(d["handle"])
    wrong = xs[3].clone()
    wrong[100] ^= 1
    assert srv.wait(srv.submit_decode(res[3]["handle"], expect=wrong))["status"] == -9
    # replay: every request checked, every result discarded
    rng = np.random.default_rng(11)
    reqs, arr, t = [], [], 0.0
    for i in range(80):
        k = int(rng.integers(0, len(xs)))
        if rng.random() < 0.7:
            reqs.append((OP_C, xs[k], 0, want[k].data_ptr(), bits[k]))
        else:
            reqs.append((OP_D, None, res[k]["handle"], xs[k].data_ptr(), 0))
        t += float(rng.exponential(0.0003))
        arr.append(t)
    out = srv.replay(reqs, arr, discard=True)
    assert all(r["status"] == 0 for r in out)
    for r in res:
        srv.release(r["handle"])
    st = srv.stats()
    assert st["mem_used"] == 0
    srv.close()
