"""Benchmark of the MI355X Huffman codec.

One step = the whole hot path over one batch of input already resident in
HBM: byte histogram -> device codebook (tie-ruled Huffman lengths,
canonical codes, decode tables) -> chunked encode (segment index + decode
index) -> indexed decode.  `value` is input bytes per second of that whole
path (GB/s, 1e9 B/s).  Prints ONE JSON line.

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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
WORKLOADS = {
    # name: (description, chunk size, decode sub-block)
    "markov_45MiB": ("45 MiB order-2 Markov text over 96 printable bytes (Zipf(1.0) rows, newline after N(70,15)), "
                     "global codebook, 256 KiB chunks, decode index every 128 bytes", 256 << 10, 128),
    "zipf96_1MiB": ("1 MiB i.i.d. Zipf(1.1) over 96 printable bytes, 64 KiB chunks", 64 << 10, 256),
    "markov_2GiB": ("2 GiB order-2 Markov text, 1 MiB chunks", 1 << 20, 256),
    "zipf256_2GiB": ("2 GiB i.i.d. Zipf(0.8) over 256 byte values, 1 MiB chunks", 1 << 20, 256),
    "markov_1GiB": ("1 GiB order-2 Markov text (the leading 2^30 bytes of markov_2GiB), 1 MiB chunks, decode index "
                    "every 128 bytes", 1 << 20, 128),
    "zipf256_1GiB": ("1 GiB i.i.d. Zipf(0.8) over 256 byte values (the leading 2^30 bytes of zipf256_2GiB), 1 MiB "
                     "chunks, decode index every 128 bytes", 1 << 20, 128),
}
# kernel ids of huff_ctx_kernel_time -> kernel names.  "scan" times the tile
# bit counts and the offset scan together; "decode" times both staged launches
# (table-only codes, longer codes) for sub-blocks of 32..256 bytes, the direct
# kernel otherwise.
KERNEL_NAMES = {"hist": "k_hist", "codebook": "k_codebook", "scan": "k_tile_scan", "encode": "k_encode",
                "decode": "k_decode_lds"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2306_11070_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str, kernel: str, source_hash: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None if there is none or it was taken on different kernel source."""
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
    try:
        return float(kv[f"{kernel}_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(a, chunk: int, passes: int):
    """The oracle (plain serial C) over the whole workload, `passes` times."""
    import oracle

    t0 = time.perf_counter()
    for _ in range(passes):
        r = oracle.compress(a, chunk)
        out = oracle.decode(r["words"], r["chunk_off"], a.size, chunk, r["len"])
    dt = (time.perf_counter() - t0) / passes
    return r, out, dt


def batch_leg(P, codec, nfiles: int, reps: int, sub: int = 128):
    """Many files, one codebook each: the batched path (one graph replay per
    operation) against a per-file loop of plain calls with a host sync per
    file, on the same files and buffers."""
    import numpy as np
    import torch

    import datagen

    t0 = time.perf_counter()
    with ThreadPoolExecutor(16) as ex:  # one file per task: most files are a single generator block
        data = list(ex.map(lambda i: datagen.batch_file(5, i), range(nfiles)))
    total = sum(a.size for a in data)
    xs = [torch.from_numpy(a).cuda() for a in data]
    chunk = 256 << 10
    files = P.batch_buffers(codec, xs, chunk, sub, bits_per_byte=8)  # byte codes average at most 8 bits
    gen_s = time.perf_counter() - t0
    b = P.Batch(codec, files, chunk, sub)
    b.compress(graph=True)
    b.decode(graph=True)
    torch.cuda.synchronize()
    ok = all(int(f["status"].item()) == 0 for f in files) and all(torch.equal(f["out"], x) for f, x in zip(files, xs))
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
    # baseline: per-file plain calls, host sync per file
    loop = []
    for _ in range(max(1, reps // 5)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for f in files:
            c = codec.compress(f["in"], chunk, sub, out=dict(hist=f["hist"], dcb=f["cb"], words=f["words"],
                                                            chunk_off=f["chunk_off"], sub_lo=f["sub_lo"]))
            codec.decompress(c, out=f["out"])
            torch.cuda.synchronize()
        loop.append(time.perf_counter() - t)
    ok = ok and all(torch.equal(f["out"], x) for f, x in zip(files, xs))
    b.close()
    ms = float(np.median(tc)) + float(np.median(td))
    loop_s = float(np.median(loop))
    return {"workload": f"{nfiles} files, sizes log-uniform 4 KiB-16 MiB, i.i.d. Zipf(s~U[0.6,1.6]) over K~U{{16..256}} "
                        f"bytes each, one codebook per file, C={chunk}, S={sub}",
            "n_files": nfiles, "n_bytes": total, "compress_ms": round(float(np.median(tc)), 3),
            "decode_ms": round(float(np.median(td)), 3), "GBps": round(total / (ms * 1e-3) / 1e9, 2),
            "per_file_loop_GBps": round(total / loop_s / 1e9, 2), "speedup_vs_loop": round(loop_s * 1e3 / ms, 2),
            "graph": True, "roundtrip_ok": bool(ok), "datagen_s": round(gen_s, 1)}


SWEEP_CHUNKS = [16 << 10, 32 << 10, 64 << 10, 128 << 10, 256 << 10, 512 << 10, 1 << 20, 2 << 20, 4 << 20]


def sweep_leg(P, codec, x, n: int, sub: int, reps: int):
    """Compress and decode times over chunk sizes 16 KiB-4 MiB, with the
    sub-block index and with the chunk index alone (decode parallelism is
    then one lane per chunk); HIP events on the current stream, median of
    `reps`.  The stream does not depend on the chunk size, only the index."""
    import torch

    def med(fn):
        ts = []
        for _ in range(reps + 1):
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


def _dev_equal(pa: int, pb: int, nbytes: int) -> bool:
    """Compares two device byte ranges (copies both to the host)."""
    import ctypes

    import numpy as np
    import torch

    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    a, b = np.empty(nbytes, np.uint8), np.empty(nbytes, np.uint8)
    torch.cuda.synchronize()
    if nbytes and (hip.hipMemcpy(a.ctypes.data, pa, nbytes, 2) or hip.hipMemcpy(b.ctypes.data, pb, nbytes, 2)):
        return False
    return bool(np.array_equal(a, b))


def serve_leg(P, seconds: float, pool_n: int, rates):
    """Open-loop serving: Poisson arrivals at fractions of the saturation
    rate, 70 % compress / 30 % decompress of resident streams, request sizes
    log-uniform 1 KiB-64 MiB (Markov text), admission by a 64 GB budget."""
    import numpy as np
    import torch

    import datagen

    sizes = [datagen.file_params(6, i, size_lo=1 << 10, size_hi=64 << 20)[0] for i in range(pool_n)]
    pool = [torch.from_numpy(datagen.markov(n, 6_000_000 + i)).cuda() for i, n in enumerate(sizes)]
    mean = float(np.mean(sizes))
    srv = P.Server(mem_budget=64 << 30, nslots=2, max_batch=256, chunk_size=256 << 10, sub_size=128)
    base = [srv.wait(srv.submit_compress(x)) for x in pool]
    ref = {i: srv.stream(r["handle"]) for i, r in enumerate(base)}
    rng = np.random.default_rng(6)

    def make(count, rate):
        reqs, arr, idx, t = [], [], [], 0.0
        for _ in range(count):
            k = int(rng.integers(0, pool_n))
            if rng.random() < 0.7:
                reqs.append((0, pool[k], 0))
            else:
                reqs.append((2, None, base[k]["handle"]))
            idx.append(k)
            arr.append(t)
            t += float(rng.exponential(1.0 / rate)) if rate else 0.0
        return reqs, arr, idx

    def run(reqs, arr, keep=()):
        res = srv.replay(reqs, arr, discard=[j for j in range(len(reqs)) if j not in keep])
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        t_first = min(r["t_submit"] for r in res)
        t_last = max(r["t_done"] for r in res)
        moved = sum((r["in_bytes"] if op == 0 else r["out_bytes"]) for (op, _, _), r in zip(reqs, res))
        good = all(r["status"] == 0 for r in res)
        return res, lat, moved / (t_last - t_first) / 1e9, good

    def check_and_release(reqs, idx, res, sample):
        ok = True
        for j, ((op, x, h), k, r) in enumerate(zip(reqs, idx, res)):
            if j not in sample or r["status"] != 0:
                continue
            a = srv.stream(r["handle"])
            if op == 0:  # the served stream equals the one served alone, word for word
                bref = ref[k]
                nw = (bref["total_bits"] + 31) // 32
                ok = ok and a["total_bits"] == bref["total_bits"] and _dev_equal(a["words"], bref["words"], nw * 4)
            else:  # the decoded bytes equal the pool input
                ok = ok and _dev_equal(a["out"], pool[k].data_ptr(), pool[k].numel())
            srv.release(r["handle"])
        return ok

    # saturation: the whole burst at t = 0
    reqs, arr, idx = make(min(2000, 8 * pool_n), 0)
    res, lat, thr, good = run(reqs, arr)
    lam_sat = thr * 1e9 / mean
    out = {"workload": f"pool of {pool_n} Markov-text requests, sizes log-uniform 1 KiB-64 MiB (mean {mean / 1e6:.2f} MB), "
                       f"70% compress / 30% decompress, 64 GB budget, {seconds:g} s per rate",
           "saturation_GBps": round(thr, 2), "lambda_sat_per_s": round(lam_sat, 1), "rates": []}
    for f in rates:
        lam = f * lam_sat
        count = max(20, int(lam * seconds))
        reqs, arr, idx = make(count, lam)
        sample = set(rng.choice(len(reqs), size=min(100, len(reqs)), replace=False).tolist())
        res, lat, thr, good = run(reqs, arr, keep=sample)
        ok = check_and_release(reqs, idx, res, sample)
        out["rates"].append({"load": f, "lambda_per_s": round(lam, 1), "requests": count,
                             "throughput_GBps": round(thr, 2), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                             "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "all_ok": bool(good and ok)})
    st = srv.stats()
    out["batches"] = st["batches"]
    for r in base:
        srv.release(r["handle"])
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="markov_45MiB", choices=sorted(WORKLOADS))
    ap.add_argument("--sub", type=int, default=None, help="decode sub-block bytes (0: chunk index only)")
    ap.add_argument("--cpu-passes", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true", help="also run the plain copy kernel (counter calibration)")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-file batch leg")
    ap.add_argument("--batch-files", type=int, default=4096)
    ap.add_argument("--batch-sub", type=int, default=128, help="decode sub-block bytes of the batch leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-segments", action="store_true", help="skip the per-segment codebook leg")
    ap.add_argument("--segment", type=int, default=256 << 10, help="segment bytes of the per-segment codebook leg")
    ap.add_argument("--sweep", action="store_true",
                    help="also time compress and decode over chunk sizes 16 KiB-4 MiB, with and without the sub-block index")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-pool", type=int, default=384)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this codec runs on a single MI355X and multi-GPU sharding is not "
              "built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_2306_11070_amd as P

    desc, chunk, sub = WORKLOADS[args.workload]
    if args.sub is not None:
        sub = args.sub
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    codec = P.Codec(0)

    a = datagen.workload(args.workload)
    n = a.size
    x = torch.from_numpy(a).to(dev)
    hist = torch.empty(256, dtype=torch.int64, device=dev)
    dcb = torch.empty(P.DCB_BYTES, dtype=torch.uint8, device=dev)
    words = torch.empty((n + 3) // 4 + 4, dtype=torch.int32, device=dev)
    off = torch.empty((n + chunk - 1) // chunk + 1, dtype=torch.int64, device=dev)
    sub_lo = torch.empty((n + sub - 1) // sub + 1, dtype=torch.int32, device=dev) if sub else None
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)

    bufs = dict(hist=hist, dcb=dcb, words=words, chunk_off=off, sub_lo=sub_lo)

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        codec.compress(x, chunk, sub, status=status, out=bufs)
        if ev is not None:
            ev[1].record()
        codec.decode(words, words.numel(), off, n, chunk, dcb, sub_lo, sub, out=out, status=status)
        if ev is not None:
            ev[2].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.copy_probe:
        y = torch.empty_like(x)
        for _ in range(3):
            codec.copy(x, y)
        torch.cuda.synchronize()
        del y

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    # per-kernel launch durations: the same steps again, with the library
    # recording a HIP event pair around each launch on the stream the kernel
    # runs on (kept out of the pass above: each event adds a few us between
    # launches)
    codec.set_timing(True)
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    ktime = {k: codec.kernel_time(k) for k in KERNEL_NAMES}
    codec.set_timing(False)

    assert int(status.item()) == 0, f"device status {int(status.item())}"
    assert torch.equal(out, x), "decoded output differs from the input"

    phase_ms = {name: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(args.steps)]))
                for i, name in enumerate(("compress", "decode"))}
    d = P.dcb_to_host(dcb)
    T = int(d.total_bits)
    nchunks = (n + chunk - 1) // chunk
    nsub = (n + sub - 1) // sub if sub else 0
    index_bytes = 8 * (nchunks + 1) + (4 * (nsub + 1) if sub else 0)
    alg = {  # algorithmic HBM bytes per call: the histogram must read the input before the encode can
        "compress": 2 * n + T / 8 + index_bytes + P.DCB_BYTES,
        "decode": T / 8 + n + index_bytes,
    }
    ntiles = (n + (16 << 10) - 1) // (16 << 10)
    kalg = {  # algorithmic HBM bytes per launch of each kernel
        "hist": n,
        "codebook": P.DCB_BYTES,
        "scan": ntiles * (512 + 4),  # u16 tile histograms in, tile offsets out
        "encode": n + T / 8 + index_bytes,  # input in; words, segment and decode index out
        "decode": T / 8 + index_bytes + n,  # words and index in; bytes out
    }
    names = dict(KERNEL_NAMES)
    if not (sub and 32 <= sub <= 256):
        names["decode"] = "k_decode"
    kernels = {}
    for k, (ms, cnt) in ktime.items():
        avg = ms / max(1, cnt)
        kernels[names[k]] = {"launches": cnt, "avg_us": round(avg * 1e3, 2),
                             "alg_GBps": round(kalg[k] / (avg * 1e-3) / 1e9, 1) if cnt else None}
    dom = max(ktime, key=lambda k: ktime[k][0])  # largest share of the step
    avg_ms = ktime[dom][0] / max(1, ktime[dom][1])
    achieved = kalg[dom] / (avg_ms * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = read_traffic(args.workload, names[dom], src_hash)

    value = n * args.steps / wall / 1e9
    line = {
        "metric": "Huffman encode+decode input GB/s on 1 MI355X (% HBM roofline)",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n_bytes": n, "chunk_size": chunk, "sub_size": sub,
                   "bits_per_byte": round(T / n, 4), "max_code_len": int(d.max_len),
                   "index_bytes": index_bytes, "stream_over_input": round((T / 8 + index_bytes) / n, 4),
                   "step": "huff_compress (histogram + device codebook + encode) + huff_decode"},
        "phases": {p: {"ms": round(phase_ms[p], 4), "alg_GBps": round(alg[p] / (phase_ms[p] * 1e-3) / 1e9, 1)}
                   for p in phase_ms},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "alg_bytes_per_launch": round(kalg[dom]), "avg_launch_us": round(avg_ms * 1e3, 2),
                     "kernel_source_sha256": src_hash},
        "kernels": kernels,
    }
    if not args.no_cpu:
        passes = args.cpu_passes
        r, o, dt = cpu_baseline(a, chunk, passes)
        nw = r["words"].size
        bitexact = bool(np.array_equal(words[:nw].cpu().numpy().view(np.uint32), r["words"])
                        and np.array_equal(off.cpu().numpy().view(np.uint64), r["chunk_off"])
                        and np.array_equal(o, a))
        line["cpu_baseline"] = {"value": round(n / dt / 1e9, 5), "unit": "GB/s", "cores": 1, "kind": "oracle",
                                "sample": f"the whole {n}-byte workload, histogram+codebook+encode+decode, "
                                          f"{passes} passes averaged (plain serial C, one thread)"}
        line["bitexact_vs_oracle"] = bitexact
    if args.sweep:
        line["sweep"] = sweep_leg(P, codec, x, n, sub, 3)
    if not args.no_segments:
        line["segments"] = segments_leg(P, codec, x, T, args.segment, sub, 20)
    if not args.no_batch:
        line["batch"] = batch_leg(P, codec, args.batch_files, 10, args.batch_sub)
    if not args.no_serve:
        line["serving"] = serve_leg(P, args.serve_seconds, args.serve_pool, (0.25, 0.5, 0.9, 1.2))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
