"""C-ABI checks that need no GPU: the library loads, exports every function
that include/huff.h declares with a binding, struct sizes agree, argument
errors are reported before any device work, and the host codebook builder
agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2306_11070_amd as P
from paper_2306_11070_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(huff_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = P.load()
    declared = _declared()
    assert "huff_encode" in declared and "huff_decode" in declared and "huff_histogram" in declared
    for name in sorted(declared):
        assert hasattr(lib, name), f"{name} declared but not exported"
        assert name in _abi.PROTOTYPES, f"{name} has no binding"


def test_struct_sizes_match_c():
    lib = P.load()
    assert lib.huff_abi_sizeof(0) == ctypes.sizeof(_abi.HuffDcb)
    assert lib.huff_abi_sizeof(1) == ctypes.sizeof(_abi.HuffCodebook)
    assert lib.huff_abi_sizeof(2) == ctypes.sizeof(_abi.HuffParams)
    for i, cls in enumerate((_abi.HuffFile, _abi.HuffServerCfg, _abi.HuffRequest, _abi.HuffResult,
                             _abi.HuffStreamInfo), start=3):
        assert lib.huff_abi_sizeof(i) == ctypes.sizeof(cls), cls.__name__
    assert lib.huff_abi_sizeof(99) == 0


def test_strerror():
    lib = P.load()
    assert lib.huff_strerror(0) == b"ok"
    assert lib.huff_strerror(-3) == b"corrupt stream"


def test_invalid_arguments_rejected_without_device():
    lib = P.load()
    assert lib.huff_histogram(None, None, 10, None, None) == _abi.HUFF_E_INVAL
    assert lib.huff_encode(None, None, 10, None, 1024, None, 0, None, 0, None, None, None) == _abi.HUFF_E_INVAL
    assert lib.huff_decode(None, None, 0, None, 10, 1024, None, 0, None, None, None, None) == _abi.HUFF_E_INVAL
    assert lib.huff_build_codebook(None, None) == _abi.HUFF_E_INVAL
    out = ctypes.c_void_p()
    assert lib.huff_ctx_create(-1, None, ctypes.byref(out)) == _abi.HUFF_E_INVAL


def test_batch_and_server_reject_null_handles_without_device():
    lib = P.load()
    INVAL = _abi.HUFF_E_INVAL
    out = ctypes.c_void_p()
    f = (_abi.HuffFile * 1)()
    assert lib.huff_batch_create(None, f, 1, 1024, 0, ctypes.byref(out)) == INVAL
    assert lib.huff_batch_create(None, f, 1, 1024, 0, None) == INVAL
    assert lib.huff_batch_run(None, 0, 0, None) == INVAL
    assert lib.huff_compress_batch(None, None) == INVAL
    assert lib.huff_encode_batch(None, None) == INVAL
    assert lib.huff_decode_batch(None, None) == INVAL
    lib.huff_batch_destroy(None)
    cfg = _abi.HuffServerCfg(1 << 20, 2, 16, 1 << 16, 0)
    assert lib.huff_server_create(None, ctypes.byref(cfg), ctypes.byref(out)) == INVAL
    req = _abi.HuffRequest(0, 0, None, 0, 0)
    t = ctypes.c_uint64()
    r = _abi.HuffResult()
    assert lib.huff_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == INVAL
    assert lib.huff_server_poll(None, 1, ctypes.byref(r)) == INVAL
    assert lib.huff_server_wait(None, 1, ctypes.byref(r)) == INVAL
    assert lib.huff_server_stream(None, 1, None) == INVAL
    assert lib.huff_server_release(None, 1) == INVAL
    assert lib.huff_server_replay(None, None, None, 0, None) == INVAL
    st = (ctypes.c_uint64 * 6)()
    assert lib.huff_server_stats(None, st) == INVAL
    lib.huff_server_destroy(None)


def _hist_cases():
    rng = np.random.default_rng(7)
    cases = []
    for i in range(120):
        k = int(rng.integers(0, 257))
        h = np.zeros(256, dtype=np.uint64)
        if k:
            h[rng.choice(256, size=k, replace=False)] = rng.integers(1, [3, 50, 10 ** 9][i % 3], size=k)
        cases.append(h)
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    h = np.zeros(256, dtype=np.uint64)
    h[:40] = fib
    cases.append(h)
    return cases


@pytest.mark.parametrize("case", range(121))
def test_host_codebook_matches_oracle(case):
    h = _hist_cases()[case]
    cb = P.build_codebook(h)
    ln = np.frombuffer(bytes(cb.len), dtype=np.uint8)
    code = np.ctypeslib.as_array(cb.code).astype(np.uint64)
    oln = oracle.code_lengths(h)
    assert np.array_equal(ln, oln)
    assert np.array_equal(code, oracle.canonical_codes(oln))
    assert cb.nsym == int(np.count_nonzero(oln)) and cb.max_len == int(oln.max())
    assert P.encoded_bits(h, cb) == oracle.total_bits(h, oln)


def test_timing_calls_reject_null_context_without_device():
    lib = P.load()
    ms, k = ctypes.c_double(), ctypes.c_uint64()
    assert lib.huff_ctx_set_timing(None, 1) == _abi.HUFF_E_INVAL
    assert lib.huff_ctx_kernel_time(None, _abi.HUFF_K_ENCODE, ctypes.byref(ms), ctypes.byref(k), 1) == _abi.HUFF_E_INVAL
    assert set(_abi.KERNEL_IDS.values()) == set(range(5))

