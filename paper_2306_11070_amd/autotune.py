"""Autotuner for the codec's launch parameters.

Chooses, per device and workload class, the histogram privatisation depth
and workgroup count, the encode workgroups per CU, the segment (chunk) size
and the decode granularity (sub-block size, i.e. decode lanes per chunk) by
timing candidate settings on the caller's data with HIP events, and keeps
the choices in a JSON cache.  Every candidate produces the same bits (the
parameters change only how the work is split), so the tuner needs no
correctness check beyond the library's own status word.

Each phase is tuned on its own: the histogram (timed inside compress, where
it also writes the per-tile histograms) does not depend on the encode or
decode settings, the encode only on its workgroups per CU, the decode on
the sub-block size and the direct-decode workgroup size.  The chunk size is
chosen last, from the decode-index budget: the smallest chunk whose index
(8 bytes per chunk + 4 per sub-block) stays under `max_index_frac` of the
encoded payload.
"""
from __future__ import annotations

import itertools
import json
import os
import time

DEFAULT_SPACE = {
    "hist_depth": [1, 2, 4, 8, 16, 32],
    "hist_blocks_per_cu": [2, 4, 8, 16],
    "enc_blocks_per_cu": [2, 4, 16, 64, 256],
    "sub_size": [0, 32, 64, 128, 256, 512],
    "dec_block": [64, 128, 256],
    "chunk_size": [16 << 10, 32 << 10, 64 << 10, 128 << 10, 256 << 10, 512 << 10, 1 << 20, 2 << 20, 4 << 20],
}


def workload_key(device_name: str, num_cus: int, n: int, bits_per_byte: float) -> str:
    """Cache key: device, log2 size bucket and a coarse code-length class."""
    size_bucket = max(0, int(n).bit_length() - 1)
    bpb = int(round(bits_per_byte))
    return f"{device_name}|cu{num_cus}|n2^{size_bucket}|bpb{bpb}"


def index_bytes(n: int, chunk: int, sub: int) -> int:
    nch = (n + chunk - 1) // chunk
    nsub = (n + sub - 1) // sub if sub else 0
    return 8 * (nch + 1) + (4 * (nsub + 1) if sub else 0)


def pick_min(timings: dict):
    """Key with the smallest time (ties: the first in insertion order)."""
    best, bt = None, None
    for k, t in timings.items():
        if bt is None or t < bt:
            best, bt = k, t
    return best


def choose_chunk(n: int, payload_bytes: int, sub: int, chunks, max_index_frac: float) -> int:
    """Smallest chunk size whose index stays within the budget (the largest
    candidate if none does).  Smaller chunks give more decode parallelism
    when there is no sub-block index, and finer random access."""
    ok = [c for c in sorted(chunks) if c >= max(sub, 1024)
          and index_bytes(n, c, sub) <= max_index_frac * max(1, payload_bytes)]
    return ok[0] if ok else max(chunks)


class Cache:
    def __init__(self, path: str | None = None):
        self.path = path or os.environ.get("HUFF_TUNE_CACHE",
                                            os.path.join(os.path.expanduser("~"), ".cache", "huff_autotune.json"))
        self.data = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, value: dict):
        self.data[key] = value
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def _time_ms(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def _kernel_ms(codec, kernel: str, fn, reps: int) -> float:
    """Median time of one kernel's launches inside `fn`, from the context's
    HIP events around them."""
    import torch
    fn()
    torch.cuda.synchronize()
    codec.set_timing(True)
    codec.kernel_time(kernel)  # clears
    ts = []
    for _ in range(reps):
        fn()
        torch.cuda.synchronize()
        ms, k = codec.kernel_time(kernel)
        ts.append(ms / max(1, k))
    codec.set_timing(False)
    ts.sort()
    return ts[len(ts) // 2]


def tune(x, space: dict | None = None, reps: int = 5, max_index_frac: float = 0.08, cache: Cache | None = None,
         use_cache: bool = True, device: int = 0) -> dict:
    """Tunes on the device tensor `x` (uint8).  Returns the chosen settings
    with the measured times; stores them in the cache."""
    import torch

    import paper_2306_11070_amd as P

    sp = dict(DEFAULT_SPACE)
    sp.update(space or {})
    props = torch.cuda.get_device_properties(device)
    ncu = props.multi_processor_count
    cache = cache or Cache()
    n = x.numel()
    probe = P.Codec(device)
    base = probe.compress(x, 1 << 20)
    torch.cuda.synchronize()
    T = int(P.dcb_to_host(base["dcb"]).total_bits)
    bpb = T / max(1, n)
    key = workload_key(props.name, ncu, n, bpb)
    if use_cache and cache.get(key):
        probe.close()
        return cache.get(key)
    t_start = time.time()
    result = {"key": key, "n": n, "bits_per_byte": bpb}

    # histogram: depth x workgroups, timed inside compress (where it also
    # writes the per-tile histograms the encoder's offsets come from), from
    # the context's own events around the histogram launch
    ht = {}
    cout = dict(hist=torch.empty(256, dtype=torch.int64, device=x.device),
                dcb=torch.empty(P.DCB_BYTES, dtype=torch.uint8, device=x.device),
                words=torch.empty((n + 3) // 4 + 8, dtype=torch.int32, device=x.device),
                chunk_off=torch.empty((n >> 20) + 2, dtype=torch.int64, device=x.device))
    for d, b in itertools.product(sp["hist_depth"], sp["hist_blocks_per_cu"]):
        c = P.Codec(device, dict(hist_depth=d, hist_blocks=b * ncu))
        ht[(d, b)] = _kernel_ms(c, "hist", lambda: c.compress(x, 1 << 20, out=cout), reps)
        c.close()
    del cout
    (hd, hb) = pick_min(ht)
    result.update(hist_depth=hd, hist_blocks=hb * ncu, hist_ms=ht[(hd, hb)])

    # encode: workgroups per CU (codebook fixed, from the probe)
    et = {}
    words = torch.empty((n + 3) // 4 + 8, dtype=torch.int32, device=x.device)
    off = torch.empty((n + 1023) // 1024 + 2, dtype=torch.int64, device=x.device)
    for e in sp["enc_blocks_per_cu"]:
        c = P.Codec(device, dict(enc_blocks_per_cu=e))
        et[e] = _time_ms(lambda: c.encode(x, base["dcb"], 1 << 20, 0, words=words, chunk_off=off), reps)
        c.close()
    eb = pick_min(et)
    result.update(enc_blocks_per_cu=eb, encode_ms=et[eb])

    # decode: sub-block size x direct-decode workgroup size, under the index budget
    dt = {}
    outb = torch.empty(n, dtype=torch.uint8, device=x.device)
    for s in sp["sub_size"]:
        chunk = max(1 << 20, s)
        if s and index_bytes(n, chunk, s) > max_index_frac * max(1, T // 8):
            continue
        cc = probe.compress(x, chunk, s)
        for db in sp["dec_block"]:
            c = P.Codec(device, dict(dec_block=db))
            dt[(s, db)] = _time_ms(lambda: c.decompress(cc, out=outb), reps)
            c.close()
    (sb, db) = pick_min(dt)
    result.update(sub_size=sb, dec_block=db, decode_ms=dt[(sb, db)])
    result["chunk_size"] = choose_chunk(n, T // 8, sb, sp["chunk_size"], max_index_frac)
    result["tune_seconds"] = time.time() - t_start
    result["candidates"] = {"hist": {f"{k[0]}x{k[1]}": v for k, v in ht.items()},
                            "encode": {str(k): v for k, v in et.items()},
                            "decode": {f"{k[0]}/{k[1]}": v for k, v in dt.items()}}
    probe.close()
    cache.put(key, result)
    return result


def params_of(tuned: dict) -> dict:
    """The huff_params fields of a tuning result."""
    return {k: tuned[k] for k in ("hist_blocks", "hist_depth", "dec_block", "enc_blocks_per_cu")}
