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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
WORKLOADS = {
    # name: (description, chunk size, decode sub-block)
    "markov_45MiB": ("45 MiB order-2 Markov text over 96 printable bytes (Zipf(1.0) rows, newline after N(70,15)), "
                     "global codebook, 256 KiB chunks", 256 << 10, 256),
    "zipf96_1MiB": ("1 MiB i.i.d. Zipf(1.1) over 96 printable bytes, 64 KiB chunks", 64 << 10, 256),
    "markov_2GiB": ("2 GiB order-2 Markov text, 1 MiB chunks", 1 << 20, 256),
    "zipf256_2GiB": ("2 GiB i.i.d. Zipf(0.8) over 256 byte values, 1 MiB chunks", 1 << 20, 256),
}
KERNELS = {"compress": "k_hist+k_codebook+k_encode", "decode": "k_decode_staged"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="markov_45MiB", choices=sorted(WORKLOADS))
    ap.add_argument("--sub", type=int, default=None, help="decode sub-block bytes (0: chunk index only)")
    ap.add_argument("--cpu-passes", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true", help="also run the plain copy kernel (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this codec runs on a single MI355X; multi-GPU sharding is not built "
              "(see DESIGN.md). Run with --gpus 1.", file=sys.stderr)
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
    dom = max(alg, key=lambda p: phase_ms[p])
    achieved = alg[dom] / (phase_ms[dom] * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = read_traffic(args.workload, KERNELS[dom], src_hash)

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
                   "step": "huff_compress (histogram + device codebook + encode) + huff_decode"},
        "phases": {p: {"ms": round(phase_ms[p], 4), "alg_GBps": round(alg[p] / (phase_ms[p] * 1e-3) / 1e9, 1)}
                   for p in phase_ms},
        "roofline": {"bound": "hbm", "kernel": KERNELS[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic)},
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
