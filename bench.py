"""Benchmark of the MI355X Huffman codec.

One step = the whole hot path over one batch of input already resident in
HBM: byte histogram -> device codebook (tie-ruled Huffman lengths,
canonical codes, decode tables) -> chunked encode (segment index + decode
index) -> indexed decode.  A 512 MiB buffer is written between steps, so
every step reads its input and stream from HBM, not from the caches.
`value` is input bytes per second of that whole path (GB/s, 1e9 B/s) from
HIP events around each step.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Huffman encode+decode input GB/s on 1 MI355X (% HBM roofline); serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
WORKLOADS = {
    # name: (description, chunk size, decode sub-block) -- the autotuner may replace chunk and sub-block
    "markov_1GiB": ("1 GiB order-2 Markov text over 96 printable bytes (the leading 2^30 bytes of the 2 GiB "
                    "Markov stream), global codebook", 1 << 20, 128),
    "zipf256_1GiB": ("1 GiB i.i.d. Zipf(0.8) over 256 byte values (the leading 2^30 bytes of the 2 GiB Zipf "
                     "stream), global codebook", 1 << 20, 128),
    "markov_45MiB": ("45 MiB order-2 Markov text over 96 printable bytes (Zipf(1.0) rows, newline after N(70,15)), "
                     "global codebook", 256 << 10, 64),
    "zipf96_1MiB": ("1 MiB i.i.d. Zipf(1.1) over 96 printable bytes", 64 << 10, 256),
}
# the 2 GiB streams stay off the GPU: a run of that case once ended in a GPU
# memory fault whose cause has not been shown
REFUSED = {"markov_2GiB", "zipf256_2GiB"}
# kernel ids of huff_ctx_kernel_time -> kernel names.  "scan" times the tile
# bit counts and the offset scans together; "decode" times the staged
# decoder's launches for sub-blocks of 32..256 bytes, the direct kernel
# otherwise.
KERNEL_NAMES = {"hist": "k_hist", "codebook": "k_codebook", "scan": "k_tile_scan", "encode": "k_encode",
                "decode": "k_decode_lds"}
TUNE_SPACE = {"hist_depth": [8, 16, 32], "hist_blocks_per_cu": [4, 16], "enc_blocks_per_cu": [4, 16, 256],
              "sub_size": [64, 128, 256], "dec_block": [256]}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2306_11070_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def progress(msg: str):
    """One line on stderr when a part of a long run ends."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def read_traffic(workload: str, kernel: str, source_hash: str, chunk: int, sub: int):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None if there is none or it was taken on different kernel source or with
    other chunk or sub-block sizes."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != source_hash:
        return None
    if kv.get("chunk_size") != str(chunk) or kv.get("sub_size") != str(sub):
        return None
    try:
        return float(kv[f"{kernel}_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(a, chunk: int) -> dict:
    """The oracle (plain serial C, one thread) phase by phase on `a`."""
    import numpy as np

    import oracle

    t = {}
    t0 = time.perf_counter()
    h = oracle.histogram(a)
    t["hist"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    ln = oracle.code_lengths(h)
    cd = oracle.canonical_codes(ln)
    t["codebook"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    w, off = oracle.encode(a, ln, cd, chunk)
    t["encode"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    out = oracle.decode(w, off, a.size, chunk, ln)
    t["decode"] = time.perf_counter() - t0
    assert np.array_equal(out, a)
    total = sum(t.values())
    return {"value": round(a.size / total / 1e9, 5), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the leading {a.size} bytes of the workload, histogram+codebook+encode+decode, one pass "
                      f"(plain serial C, one thread)",
            "phase_s": {k: round(v, 3) for k, v in t.items()},
            "phase_GBps": {k: round(a.size / v / 1e9, 4) for k, v in t.items() if v > 0}, **host_info()}


class Flusher:
    """Writes a buffer larger than the L2 and Infinity Cache between steps."""

    def __init__(self, mib: int):
        import torch
        self.buf = torch.empty(max(1, mib) << 20, dtype=torch.uint8, device="cuda") if mib else None
        self.k = 0

    def __call__(self):
        if self.buf is not None:
            self.k = (self.k + 1) & 0x7F
            self.buf.fill_(self.k)


def run_stream(P, codec, x, chunk: int, sub: int, steps: int, warmup: int, flush: Flusher, graph: bool = False,
               settle_s: float = 0.0):
    """Times `steps` flushed steps (compress + decode, each replayed from a HIP
    graph when `graph`) with HIP events, then the same steps again, eagerly,
    with the library's per-kernel event timing.  Before the `warmup` steps,
    untimed steps run for `settle_s` seconds: launch times fall over the
    first tens of milliseconds of sustained work as the GPU's clocks settle."""
    import numpy as np
    import torch

    n = x.numel()
    dev = x.device
    bufs = dict(hist=torch.empty(256, dtype=torch.int64, device=dev),
                dcb=torch.empty(P.DCB_BYTES, dtype=torch.uint8, device=dev),
                words=torch.empty((n + 3) // 4 + 4, dtype=torch.int32, device=dev),
                chunk_off=torch.empty((n + chunk - 1) // chunk + 1, dtype=torch.int64, device=dev),
                sub_lo=torch.empty((n + sub - 1) // sub + 1, dtype=torch.int32, device=dev) if sub else None)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)

    def compress():
        codec.compress(x, chunk, sub, status=status, out=bufs)

    def decode():
        codec.decode(bufs["words"], bufs["words"].numel(), bufs["chunk_off"], n, chunk, bufs["dcb"],
                     bufs["sub_lo"], sub, out=out, status=status)

    def step(ev=None, run_c=compress, run_d=decode):
        flush()
        if ev is not None:
            ev[0].record()
        run_c()
        if ev is not None:
            ev[1].record()
        run_d()
        if ev is not None:
            ev[2].record()

    settle_steps = 0
    t_settle = time.perf_counter() + settle_s
    while time.perf_counter() < t_settle:
        step()
        torch.cuda.synchronize()
        settle_steps += 1
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    run_c, run_d = compress, decode
    if graph:
        # each call's launches captured once into a HIP graph and replayed
        # (the context's workspaces are sized by the eager warm-up steps)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        gc, gd = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(gc, stream=s):
                compress()
            with torch.cuda.graph(gd, stream=s):
                decode()
        torch.cuda.synchronize()
        run_c, run_d = gc.replay, gd.replay
        step(None, run_c, run_d)
        torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k], run_c, run_d)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    comp = [evs[k][0].elapsed_time(evs[k][1]) for k in range(steps)]
    dec = [evs[k][1].elapsed_time(evs[k][2]) for k in range(steps)]
    # per-kernel launch durations: the same steps again, the library recording
    # an event pair around each launch on the stream the kernel runs on (kept
    # out of the pass above: each event pair adds a few us between launches)
    codec.set_timing(True)
    for _ in range(steps):
        step(None, compress, decode)
    torch.cuda.synchronize()
    ktime = {k: codec.kernel_time(k) for k in KERNEL_NAMES}
    codec.set_timing(False)
    assert int(status.item()) == 0, f"device status {int(status.item())}"
    assert torch.equal(out, x), "decoded output differs from the input"
    return {"compress_ms": float(np.mean(comp)), "decode_ms": float(np.mean(dec)), "wall_s": wall,
            "settle_steps": settle_steps,
            "ktime": ktime, "bufs": bufs, "out": out}


def stream_report(P, n: int, chunk: int, sub: int, r: dict, workload: str) -> dict:
    """Per-phase and per-kernel algorithmic GB/s and HBM roofline fractions."""
    d = P.dcb_to_host(r["bufs"]["dcb"])
    T = int(d.total_bits)
    nchunks = (n + chunk - 1) // chunk
    nsub = (n + sub - 1) // sub if sub else 0
    index_bytes = 8 * (nchunks + 1) + (4 * (nsub + 1) if sub else 0)
    ntiles = (n + (16 << 10) - 1) // (16 << 10)
    kalg = {  # algorithmic HBM bytes per launch of each kernel
        "hist": n,  # input in (per-tile u16 histograms are workspace, counted under scan)
        "codebook": P.DCB_BYTES,
        "scan": ntiles * (512 + 4),  # u16 tile histograms in, tile offsets out
        "encode": n + T / 8 + index_bytes,  # input in; words, segment and decode index out
        "decode": T / 8 + index_bytes + n,  # words and index in; bytes out
    }
    names = dict(KERNEL_NAMES)
    if not (sub and 32 <= sub <= 256):
        names["decode"] = "k_decode"
    kernels = {}
    for k, (ms, cnt) in r["ktime"].items():
        avg = ms / max(1, cnt)
        ach = kalg[k] / (avg * 1e-3) / 1e9 if cnt else None
        kernels[names[k]] = {"launches": cnt, "avg_us": round(avg * 1e3, 2),
                             "alg_bytes_per_launch": round(kalg[k]),
                             "alg_GBps": None if ach is None else round(ach, 1),
                             "frac": None if ach is None else round(ach / HBM_PEAK_GBS, 4)}
    dom = max(r["ktime"], key=lambda k: r["ktime"][k][0])  # largest share of the step
    avg_ms = r["ktime"][dom][0] / max(1, r["ktime"][dom][1])
    achieved = kalg[dom] / (avg_ms * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = read_traffic(workload, names[dom], src_hash, chunk, sub)
    step_ms = r["compress_ms"] + r["decode_ms"]
    alg = {"compress": 2 * n + T / 8 + index_bytes + P.DCB_BYTES, "decode": T / 8 + n + index_bytes}
    return {
        "T": T, "max_len": int(d.max_len), "index_bytes": index_bytes, "step_ms": step_ms,
        "phases": {"compress": {"ms": round(r["compress_ms"], 4),
                                "alg_GBps": round(alg["compress"] / (r["compress_ms"] * 1e-3) / 1e9, 1)},
                   "decode": {"ms": round(r["decode_ms"], 4),
                              "alg_GBps": round(alg["decode"] / (r["decode_ms"] * 1e-3) / 1e9, 1)}},
        "phase_roofline": {p: kernels[names[p]]["frac"] for p in ("hist", "encode", "decode")},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "alg_bytes_per_launch": round(kalg[dom]), "avg_launch_us": round(avg_ms * 1e3, 2),
                     "kernel_source_sha256": src_hash},
        "kernels": kernels,
    }


def copy_probe(codec, src, dst, flush: Flusher, reps: int = 5) -> dict:
    """The plain copy kernel over the same bytes: what a kernel that only
    moves data reaches on this device (median of `reps`, flushed)."""
    import numpy as np
    import torch

    n = src.numel()
    ts = []
    for _ in range(reps + 1):
        flush()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        codec.copy(src, dst, n)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts[1:]))
    gbs = 2 * n / (ms * 1e-3) / 1e9
    assert torch.equal(src, dst)
    return {"bytes_moved": 2 * n, "ms": round(ms, 4), "GBps": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def oracle_check(a, r: dict, chunk: int, sub: int) -> dict:
    """Every word, chunk offset and sub-block offset of the GPU stream against
    the oracle (piece by piece on the host cores)."""
    import numpy as np

    import oracle
    from oracle import pieces

    t0 = time.perf_counter()
    b = r["bufs"]
    h = b["hist"].cpu().numpy().view(np.uint64)
    ok = bool(np.array_equal(h, np.bincount(a, minlength=256).astype(np.uint64)))
    ln = oracle.code_lengths(h)
    cd = oracle.canonical_codes(ln)
    T = oracle.total_bits(h, ln)
    words = b["words"][:(T + 31) // 32].cpu().numpy().view(np.uint32)
    off = b["chunk_off"].cpu().numpy().view(np.uint64)
    sl = b["sub_lo"].cpu().numpy().view(np.uint32) if sub else None
    try:
        ok = ok and pieces.check_stream(a, words, off, sl, ln, cd, chunk, sub) == T
    except AssertionError:
        ok = False
    return {"bitexact_vs_oracle": ok, "check_s": round(time.perf_counter() - t0, 1),
            "checked": "histogram, every word, every chunk offset and sub-block offset; decode equals the input"}


def tune_leg(x, cache_path: str) -> dict:
    from paper_2306_11070_amd import autotune as A

    cache = A.Cache(cache_path)
    return A.tune(x, space=TUNE_SPACE, reps=3, cache=cache, use_cache=False)


def batch_leg(P, params: dict, nfiles: int, reps: int, chunk: int, sub: int):
    """Many files, one codebook each: the batched path (one graph replay per
    operation) against a per-file loop of plain calls with a host sync per
    file, on the same files and buffers; then every file against the oracle
    on that file alone, in a thread pool over the host cores."""
    import numpy as np
    import torch

    import datagen
    import oracle

    codec = P.Codec(0, params)
    t0 = time.perf_counter()
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:  # one file per task: most files are a single generator block
        data = list(ex.map(lambda i: datagen.batch_file(5, i), range(nfiles)))
    total = sum(a.size for a in data)
    xs = [torch.from_numpy(a).cuda() for a in data]
    files = P.batch_buffers(codec, xs, chunk, sub, bits_per_byte=8)  # byte codes average at most 8 bits
    gen_s = time.perf_counter() - t0
    b = P.Batch(codec, files, chunk, sub)
    b.compress(graph=True)
    b.decode(graph=True)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tc, td = [], []
    for _ in range(reps):
        ev[0].record()
        b.compress(graph=True)
        ev[1].record()
        b.decode(graph=True)
        ev[2].record()
        torch.cuda.synchronize()
        tc.append(ev[0].elapsed_time(ev[1]))
        td.append(ev[1].elapsed_time(ev[2]))
    ok = all(int(f["status"].item()) == 0 for f in files) and all(torch.equal(f["out"], x) for f, x in zip(files, xs))
    # the oracle on every file alone: words and segment index
    words = [f["words"] for f in files]
    offs = [f["chunk_off"].cpu().numpy().view(np.uint64) for f in files]

    def check(i):
        r = oracle.compress(data[i], chunk)
        w = words[i][: r["words"].size].cpu().numpy().view(np.uint32)
        return bool(np.array_equal(w, r["words"]) and np.array_equal(offs[i], r["chunk_off"]))

    t1 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:
        oracle_ok = all(ex.map(check, range(nfiles)))
    oracle_s = time.perf_counter() - t1
    # baseline: per-file plain calls, host sync per file
    loop = []
    for _ in range(max(1, reps // 5)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for f in files:
            c = codec.compress(f["in"], chunk, sub, out=dict(hist=f["hist"], dcb=f["cb"], words=f["words"],
                                                            chunk_off=f["chunk_off"], sub_lo=f.get("sub_lo")))
            codec.decompress(c, out=f["out"])
            torch.cuda.synchronize()
        loop.append(time.perf_counter() - t)
    ok = ok and all(torch.equal(f["out"], x) for f, x in zip(files, xs))
    b.close()
    codec.close()
    ms = float(np.median(tc)) + float(np.median(td))
    loop_s = float(np.median(loop))
    return {"workload": f"{nfiles} files, sizes log-uniform 4 KiB-16 MiB, i.i.d. Zipf(s~U[0.6,1.6]) over K~U{{16..256}} "
                        f"bytes each, one codebook per file",
            "chunk_size": chunk, "sub_size": sub, "params": params,
            "n_files": nfiles, "n_bytes": total, "compress_ms": round(float(np.median(tc)), 3),
            "decode_ms": round(float(np.median(td)), 3), "GBps": round(total / (ms * 1e-3) / 1e9, 2),
            "per_file_loop_GBps": round(total / loop_s / 1e9, 2), "speedup_vs_loop": round(loop_s * 1e3 / ms, 2),
            "graph": True, "roundtrip_ok": bool(ok), "bitexact_vs_oracle_every_file": bool(oracle_ok),
            "cpu_baseline": {"value": round(total / oracle_s / 1e9, 4), "unit": "GB/s", "cores": workers,
                             "kind": "oracle", "sample": f"all {nfiles} files, histogram+codebook+encode per file, "
                                                         f"one file per task in a pool of {workers} threads"},
            "datagen_s": round(gen_s, 1)}


SWEEP_CHUNKS = [16 << 10, 32 << 10, 64 << 10, 128 << 10, 256 << 10, 512 << 10, 1 << 20, 2 << 20, 4 << 20]


def sweep_leg(P, codec, x, n: int, sub: int, reps: int, flush: Flusher):
    """Compress and decode times over chunk sizes 16 KiB-4 MiB, with the
    sub-block index and with the chunk index alone (decode parallelism is
    then one lane per chunk); HIP events, flushed, median of `reps`."""
    import torch

    def med(fn):
        ts = []
        for _ in range(reps + 1):
            flush()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts = sorted(ts[1:])
        return ts[len(ts) // 2]

    rows = []
    out = torch.empty(n, dtype=torch.uint8, device=x.device)
    for chunk in SWEEP_CHUNKS:
        for s in (sub, 0):
            st = codec.new_status()
            c = codec.compress(x, chunk, s, status=st)
            cms = med(lambda: codec.compress(x, chunk, s, status=st, out=c))
            dms = med(lambda: codec.decompress(c, out=out, status=st))
            torch.cuda.synchronize()
            ok = int(st.item()) == 0 and bool(torch.equal(out, x))
            rows.append({"chunk": chunk, "sub": s, "compress_ms": round(cms, 4), "decode_ms": round(dms, 4),
                         "compress_GBps": round(n / (cms * 1e-3) / 1e9, 1),
                         "decode_GBps": round(n / (dms * 1e-3) / 1e9, 1), "roundtrip_ok": ok})
            del c
    return rows


def segments_leg(P, codec, x, T_global: int, seg: int, sub: int, reps: int):
    """The same input with a codebook per segment (one batch plan over the
    segments, graph replays), against the global codebook's size."""
    import numpy as np
    import torch

    sg = P.Segments(codec, x, seg, seg, sub)
    sg.compress(graph=True)
    sg.decode(graph=True)
    torch.cuda.synchronize()
    ok = all(int(v) == 0 for v in sg.status.cpu().tolist()) and bool(torch.equal(sg.out, x))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tc, td = [], []
    for _ in range(reps):
        ev[0].record()
        sg.compress(graph=True)
        ev[1].record()
        sg.decode(graph=True)
        ev[2].record()
        torch.cuda.synchronize()
        tc.append(ev[0].elapsed_time(ev[1]))
        td.append(ev[1].elapsed_time(ev[2]))
    bits = sum(sg.segment_bits())
    n = x.numel()
    ms = float(np.median(tc)) + float(np.median(td))
    # stored size: payload plus the 256 code lengths of each codebook
    size_seg = bits / 8 + 256 * sg.nseg
    size_glb = T_global / 8 + 256
    sg.close()
    return {"segment_bytes": seg, "n_segments": sg.nseg, "compress_ms": round(float(np.median(tc)), 4),
            "decode_ms": round(float(np.median(td)), 4), "GBps": round(n / (ms * 1e-3) / 1e9, 2),
            "bits_per_byte": round(bits / n, 4), "size_vs_global_codebook": round(size_seg / size_glb, 5),
            "graph": True, "roundtrip_ok": ok}


def method3_leg(P, params: dict, workload: str, block: int, every: int, chunk: int, sub: int, steps: int,
                flush: Flusher, check: bool):
    """Method 3 (block transform + move-to-front + Huffman code) on one
    workload: per-phase HIP-event times (flushed), size against the plain
    Huffman code, and (check) every output against the oracle."""
    import numpy as np
    import torch

    import datagen

    codec = P.Codec(0, params)
    a = datagen.workload(workload)
    n = a.size
    x = torch.from_numpy(a).cuda()
    dev = x.device
    o = dict(last=torch.empty(n, dtype=torch.uint8, device=dev),
             rows=torch.empty(max(1, (n + every - 1) // every), dtype=torch.int16, device=dev),
             mtf=torch.empty(n, dtype=torch.uint8, device=dev),
             hist=torch.empty(256, dtype=torch.int64, device=dev),
             dcb=torch.empty(P.DCB_BYTES, dtype=torch.uint8, device=dev),
             words=torch.empty((n + 3) // 4 + 4, dtype=torch.int32, device=dev),
             chunk_off=torch.empty((n + chunk - 1) // chunk + 1, dtype=torch.int64, device=dev),
             sub_lo=torch.empty((n + sub - 1) // sub + 1, dtype=torch.int32, device=dev))
    w = dict(mtf=torch.empty(n, dtype=torch.uint8, device=dev), last=torch.empty(n, dtype=torch.uint8, device=dev))
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    names = ("bwt", "mtf", "huffman_compress", "huffman_decode", "unmtf", "unbwt")
    times = {k: [] for k in names}
    for it in range(steps + 2):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
        flush()
        ev[0].record()
        codec.bwt(x, block, every, last=o["last"], rows=o["rows"])
        ev[1].record()
        codec.mtf(o["last"], block, out=o["mtf"])
        ev[2].record()
        c = codec.compress(o["mtf"], chunk, sub, status=st, out=o)
        ev[3].record()
        codec.decompress(c, out=w["mtf"], status=st)
        ev[4].record()
        codec.unmtf(w["mtf"], block, out=w["last"])
        ev[5].record()
        codec.unbwt(w["last"], block, every, o["rows"], out=out, status=st)
        ev[6].record()
        torch.cuda.synchronize()
        if it >= 2:
            for i, k in enumerate(names):
                times[k].append(ev[i].elapsed_time(ev[i + 1]))
    ok = int(st.item()) == 0 and bool(torch.equal(out, x))
    T3 = int(c["chunk_off"][-1].item())
    plain = codec.compress(x, chunk, sub)
    T1 = int(plain["chunk_off"][-1].item())
    ms = {k: float(np.mean(v)) for k, v in times.items()}
    comp_ms = ms["bwt"] + ms["mtf"] + ms["huffman_compress"]
    dec_ms = ms["huffman_decode"] + ms["unmtf"] + ms["unbwt"]
    res = {"workload": f"{workload}, blocks of {block} bytes, a row every {every} bytes, chunks of {chunk}, "
                       f"decode index every {sub} bytes",
           "n_bytes": n, "phase_ms": {k: round(v, 4) for k, v in ms.items()},
           "phase_GBps": {k: round(n / (v * 1e-3) / 1e9, 2) for k, v in ms.items()},
           "compress_GBps": round(n / (comp_ms * 1e-3) / 1e9, 2), "decode_GBps": round(n / (dec_ms * 1e-3) / 1e9, 2),
           "GBps": round(n / ((comp_ms + dec_ms) * 1e-3) / 1e9, 2),
           "bits_per_byte": round(T3 / n, 4), "plain_huffman_bits_per_byte": round(T1 / n, 4),
           "size_vs_plain_huffman": round((T3 / 8 + 2 * ((n + every - 1) // every)) / (T1 / 8), 4),
           "bound": "alu", "roundtrip_ok": ok}
    if check:
        import oracle
        t0 = time.perf_counter()
        r = oracle.compress_bwt(a, block, every, chunk, sub)
        t1 = time.perf_counter()
        nw = r["words"].size
        res["bitexact_vs_oracle"] = bool(
            np.array_equal(o["last"].cpu().numpy(), r["last"])
            and np.array_equal(o["rows"].cpu().numpy().view(np.uint16).astype(np.uint32), r["rows"])
            and np.array_equal(o["words"][:nw].cpu().numpy().view(np.uint32), r["words"])
            and np.array_equal(o["chunk_off"].cpu().numpy().view(np.uint64), r["chunk_off"]))
        res["cpu_baseline"] = {"value": round(n / (t1 - t0) / 1e9, 5), "unit": "GB/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole {n}-byte workload, transform + move-to-front + Huffman compress "
                                         f"(plain serial C, one thread)"}
    codec.close()
    return res


def serve_leg(P, params: dict, seconds: float, pool_n: int, loads, chunk: int, sub: int):
    """Open-loop serving: Poisson arrivals at fractions of the saturation
    rate, 70 % compress / 30 % decompress of resident streams, request sizes
    log-uniform 1 KiB-64 MiB (Markov text, a seed per request), admission by
    a 64 GB budget.  Every request carries the oracle's result for its input,
    which the server compares on the device."""
    import numpy as np
    import torch

    import datagen
    import oracle

    sizes = [datagen.file_params(6, i, size_lo=1 << 10, size_hi=64 << 20)[0] for i in range(pool_n)]
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        host = list(ex.map(lambda i: datagen.markov(sizes[i], 6_000_000 + i), range(pool_n)))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:
        refs = list(ex.map(lambda a: oracle.compress(a, chunk), host))
    oracle_s = time.perf_counter() - t0
    pool = [torch.from_numpy(a).cuda() for a in host]
    want = [torch.from_numpy(np.concatenate([r["words"], np.zeros(4, np.uint32)]).view(np.int32)).cuda()
            for r in refs]
    bits = [int(r["total_bits"]) for r in refs]
    mean = float(np.mean(sizes))
    srv = P.Server(mem_budget=64 << 30, nslots=2, max_batch=256, chunk_size=chunk, sub_size=sub, params=params)
    base = [srv.wait(srv.submit_compress(x, expect=w, expect_bits=b)) for x, w, b in zip(pool, want, bits)]
    assert all(r["status"] == 0 for r in base)
    rng = np.random.default_rng(6)

    in_ptr = np.array([x.data_ptr() for x in pool], dtype=np.uint64)
    in_n = np.array([x.numel() for x in pool], dtype=np.uint64)
    want_ptr = np.array([w.data_ptr() for w in want], dtype=np.uint64)
    want_bits = np.array(bits, dtype=np.uint64)
    handles = np.array([r["handle"] for r in base], dtype=np.uint64)

    def make(count, rate):
        k = rng.integers(0, pool_n, size=count)
        comp = rng.random(count) < 0.7
        gaps = rng.exponential(1.0 / rate, size=count) if rate else np.zeros(count)
        arr = np.concatenate([[0.0], np.cumsum(gaps)[:-1]])
        q = P.Server.request_array(count)
        q["op"] = np.where(comp, 0, 2)
        q["flags"] = 1  # HUFF_REQ_DISCARD: results are freed once checked
        q["d_in"] = np.where(comp, in_ptr[k], 0)
        q["n"] = np.where(comp, in_n[k], 0)
        q["stream_handle"] = np.where(comp, 0, handles[k])
        q["d_expect"] = np.where(comp, want_ptr[k], in_ptr[k])  # words, or the original bytes for a decode
        q["expect_bits"] = np.where(comp, want_bits[k], 0)
        return q, arr

    def run(q, arr):
        res = srv.replay_array(q, arr)
        lat = res["t_done"] - res["t_submit"]
        span = float(res["t_done"].max() - res["t_submit"].min())
        moved = float(np.where(q["op"] == 0, res["in_bytes"], res["out_bytes"]).sum())
        bad = int(np.count_nonzero(res["status"] != 0))
        return lat, moved / span / 1e9, len(res) / span, bad

    # the knee: offered rates rising from a burst's estimate; saturation is
    # the largest delivered request rate
    reqs, arr = make(min(2000, 8 * pool_n), 0)
    _, thr0, _, bad0 = run(reqs, arr)
    lam0 = thr0 * 1e9 / mean
    knee = []
    for f in (0.5, 0.75, 1.0, 1.25, 1.5, 2.0):
        lam = f * lam0
        reqs, arr = make(max(50, int(lam * min(2.0, seconds))), lam)
        lat, thr, rate, bad = run(reqs, arr)
        knee.append({"offered_per_s": round(lam, 1), "delivered_per_s": round(rate, 1), "throughput_GBps": round(thr, 2),
                     "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "mismatches": bad})
        progress(f"serve knee: offered {lam:.1f}/s delivered {rate:.1f}/s, {thr:.1f} GB/s, {bad} mismatches")
    lam_sat = max(k["delivered_per_s"] for k in knee)
    out = {"workload": f"pool of {pool_n} Markov-text requests, sizes log-uniform 1 KiB-64 MiB (mean {mean / 1e6:.2f} MB), "
                       f"70% compress / 30% decompress, 64 GB budget, {seconds:g} s per rate; every request's result "
                       f"compared on the device with the oracle's (words and length, or decoded bytes)",
           "chunk_size": chunk, "sub_size": sub, "oracle_pool_s": round(oracle_s, 1), "oracle_cores": workers,
           "burst_GBps": round(thr0, 2), "knee": knee, "lambda_sat_per_s": round(lam_sat, 1),
           "saturation_GBps": round(lam_sat * mean / 1e9, 2), "rates": []}
    all_ok = bad0 == 0 and all(k["mismatches"] == 0 for k in knee)
    for f in loads:
        lam = f * lam_sat
        count = max(20, int(lam * seconds))
        reqs, arr = make(count, lam)
        lat, thr, rate, bad = run(reqs, arr)
        all_ok = all_ok and bad == 0
        out["rates"].append({"load": f, "lambda_per_s": round(lam, 1), "requests": count,
                             "throughput_GBps": round(thr, 2), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                             "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "mismatches": bad,
                             "all_ok": bad == 0})
        progress(f"serve load {f}: {count} requests, {thr:.1f} GB/s, p50 {np.percentile(lat, 50) * 1e3:.2f} ms, "
                 f"p99 {np.percentile(lat, 99) * 1e3:.2f} ms, {bad} mismatches")
    st = srv.stats()
    out["batches"] = st["batches"]
    out["all_ok"] = bool(all_ok)
    for r in base:
        srv.release(r["handle"])
    srv.close()
    # the same request mix through a loop of plain calls (huff_compress or
    # huff_decode per request, a host synchronisation after each)
    codec = P.Codec(0, params)
    streams = [codec.compress(x, chunk, sub) for x in pool]
    torch.cuda.synchronize()
    nloop = min(4000, 10 * pool_n)
    k = rng.integers(0, pool_n, size=nloop)
    comp = rng.random(nloop) < 0.7
    moved = 0
    t0 = time.perf_counter()
    for i in range(nloop):
        if comp[i]:
            codec.compress(pool[k[i]], chunk, sub)
        else:
            codec.decompress(streams[k[i]])
        torch.cuda.synchronize()
        moved += sizes[k[i]]
    loop_s = time.perf_counter() - t0
    out["plain_loop"] = {"requests": nloop, "GBps": round(moved / loop_s / 1e9, 2),
                         "what": "the same 70/30 request mix, one plain huff_compress or huff_decode call per request "
                                 "with a host synchronisation after each"}
    out["saturation_vs_plain_loop"] = round(out["saturation_GBps"] / (moved / loop_s / 1e9), 2)
    del streams
    codec.close()
    progress(f"serve plain loop: {moved / loop_s / 1e9:.1f} GB/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="markov_1GiB", choices=sorted(WORKLOADS) + sorted(REFUSED))
    ap.add_argument("--chunk", type=int, default=None, help="chunk bytes (default: the autotuner's choice)")
    ap.add_argument("--sub", type=int, default=None, help="decode sub-block bytes (0: chunk index only)")
    ap.add_argument("--flush-mib", type=int, default=512, help="MiB written between steps (0: none)")
    ap.add_argument("--settle-s", type=float, default=0.3,
                    help="seconds of untimed steps before the warm-up steps, while the GPU's clocks settle (0: none)")
    ap.add_argument("--no-tune", action="store_true", help="fixed default launch parameters, no autotuning")
    ap.add_argument("--graph", action="store_true",
                    help="time each call's launches replayed from a HIP graph (measured slower than eager calls)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "gpurun_out", "autotune.json"))
    ap.add_argument("--cpu-sample-mib", type=int, default=256, help="oracle baseline on the leading MiB")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs (profiling runs)")
    ap.add_argument("--no-paper-scale", action="store_true", help="skip the 45 MiB leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-file batch leg")
    ap.add_argument("--batch-files", type=int, default=4096)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-segments", action="store_true", help="skip the per-segment codebook leg")
    ap.add_argument("--segment", type=int, default=256 << 10, help="segment bytes of the per-segment codebook leg")
    ap.add_argument("--sweep", action="store_true",
                    help="also time compress and decode over chunk sizes 16 KiB-4 MiB, with and without the sub-block index")
    ap.add_argument("--no-method3", action="store_true", help="skip the block transform (Method 3) leg")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-pool", type=int, default=384)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this codec runs on a single MI355X and multi-GPU sharding is not "
              "built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload in REFUSED:
        print(f"{args.workload}: the 2 GiB streams are not run on the GPU (a run of that case once ended in a GPU "
              "memory fault whose cause has not been shown); use markov_1GiB or zipf256_1GiB.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_2306_11070_amd as P

    desc, chunk, sub = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    a = datagen.workload(args.workload)
    n = a.size
    x = torch.from_numpy(a).to(dev)
    flush = Flusher(args.flush_mib)

    tuned = None
    params = {}
    if not args.no_tune:
        os.makedirs(os.path.dirname(args.tune_cache), exist_ok=True)
        tuned = tune_leg(x, args.tune_cache)
        from paper_2306_11070_amd import autotune as A
        params = A.params_of(tuned)
        chunk, sub = tuned["chunk_size"], tuned["sub_size"]
    if args.chunk is not None:
        chunk = args.chunk
    if args.sub is not None:
        sub = args.sub
    codec = P.Codec(0, params)
    r = run_stream(P, codec, x, chunk, sub, args.steps, args.warmup, flush, graph=args.graph, settle_s=args.settle_s)
    rep = stream_report(P, n, chunk, sub, r, args.workload)
    cp = copy_probe(codec, x, r["out"], flush)
    value = n / (rep["step_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(rep["step_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}, chunks of {chunk} bytes, decode index every {sub} bytes",
                   "n_bytes": n, "chunk_size": chunk, "sub_size": sub, "launch_params": codec.params,
                   "autotuned": tuned is not None, "bits_per_byte": round(rep["T"] / n, 4),
                   "max_code_len": rep["max_len"], "index_bytes": rep["index_bytes"],
                   "stream_over_input": round((rep["T"] / 8 + rep["index_bytes"]) / n, 4),
                   "cache": f"{args.flush_mib} MiB written between steps (not timed)",
                   "settle": f"{r['settle_steps']} untimed steps over {args.settle_s:g} s before the warm-up steps "
                             f"(launch times fall while the GPU's clocks settle)",
                   "launch": "each call's launches replayed from a HIP graph" if args.graph else "eager calls",
                   "step": "huff_compress (histogram + device codebook + encode) + huff_decode"},
        "wall_s_timed_steps_incl_flush": round(r["wall_s"], 4),
        "phases": rep["phases"],
        "phase_roofline": rep["phase_roofline"],
        "roofline": rep["roofline"],
        "copy_probe": cp,
        "kernels": rep["kernels"],
    }
    if tuned is not None:
        line["autotune"] = {k: tuned[k] for k in ("hist_depth", "hist_blocks", "enc_blocks_per_cu", "sub_size",
                                                   "dec_block", "chunk_size", "hist_ms", "encode_ms", "decode_ms",
                                                   "tune_seconds")}
        line["autotune"]["space"] = TUNE_SPACE
    T = rep["T"]
    del r["out"]
    if not args.no_cpu:
        line.update(oracle_check(a, r, chunk, sub))
        m = min(n, args.cpu_sample_mib << 20)
        line["cpu_baseline"] = cpu_baseline(a[:m], chunk)
    del r
    if args.sweep:
        line["sweep"] = sweep_leg(P, codec, x, n, sub, 3, flush)
    del x
    torch.cuda.empty_cache()
    if not args.no_paper_scale and args.workload != "markov_45MiB":
        d2, c2, s2 = WORKLOADS["markov_45MiB"]
        a2 = datagen.workload("markov_45MiB")
        x2 = torch.from_numpy(a2).to(dev)
        r2 = run_stream(P, codec, x2, c2, s2, 20, 5, flush, graph=args.graph, settle_s=args.settle_s)
        rep2 = stream_report(P, a2.size, c2, s2, r2, "markov_45MiB")
        ps = {"workload": f"markov_45MiB: {d2}, chunks of {c2} bytes, decode index every {s2} bytes",
              "value_GBps": round(a2.size / (rep2["step_ms"] * 1e-3) / 1e9, 2), "ms_per_step": round(rep2["step_ms"], 4),
              "phases": rep2["phases"], "phase_roofline": rep2["phase_roofline"], "roofline": rep2["roofline"],
              "cache": f"{args.flush_mib} MiB written between steps"}
        if not args.no_segments:
            ps["segments"] = segments_leg(P, codec, x2, rep2["T"], args.segment, s2, 20)
        line["paper_scale"] = ps
        progress("markov_45MiB leg done")
        del r2, x2
        torch.cuda.empty_cache()
    codec.close()
    if not args.no_method3:
        line["method3"] = [method3_leg(P, params, wl, 16384, 256, 256 << 10, 128, 5, flush, not args.no_cpu)
                           for wl in ("words_45MiB", "markov_45MiB")]
        progress("method 3 leg done")
        torch.cuda.empty_cache()
    if not args.no_batch:
        line["batch"] = batch_leg(P, params, args.batch_files, 10, 256 << 10, sub)
        progress("batch leg done")
        torch.cuda.empty_cache()
    if not args.no_serve:
        line["serving"] = serve_leg(P, params, args.serve_seconds, args.serve_pool,
                                    (0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2), 256 << 10, 128)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
