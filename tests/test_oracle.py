"""Pins for the CPU oracle, against facts that do not come from the oracle:
worked examples (tests/golden), Huffman theory (optimality by brute force,
closed forms, Kraft equality, the entropy bound), library routines
(numpy.bincount) and independent re-implementations of the bit layout.
Runs without a GPU."""
import itertools
import math
import os

import numpy as np
import pytest

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def _kv(s, conv=str):
    return {k: conv(v) for k, v in (p.split("=") for p in s.split())}


def _hist_of(counts: dict) -> np.ndarray:
    h = np.zeros(256, dtype=np.uint64)
    for sym, c in counts.items():
        h[ord(sym) if isinstance(sym, str) else sym] = c
    return h


def _bits(code: int, length: int) -> str:
    return format(int(code), "0{}b".format(int(length))) if length else ""


# ----------------------------------------------------------------- histogram
@pytest.mark.parametrize("n", [0, 1, 7, 4096, 100_003])
def test_histogram_matches_bincount(n):
    rng = np.random.default_rng(n)
    a = rng.integers(0, 256, size=n, dtype=np.uint8)
    assert np.array_equal(oracle.histogram(a), np.bincount(a, minlength=256).astype(np.uint64))


def test_histogram_generator_data():
    a = datagen.workload("zipf96_1MiB")
    h = oracle.histogram(a)
    assert np.array_equal(h, np.bincount(a, minlength=256).astype(np.uint64))
    assert int(h.sum()) == a.size


# ------------------------------------------------------------- code lengths
def _brute_min_cost(w):
    """Minimum of sum w_i*l_i over all length vectors with Kraft sum <= 1."""
    k = len(w)
    best = None
    for ls in itertools.product(range(1, k), repeat=k):
        if sum(2.0 ** -l for l in ls) <= 1.0 + 1e-12:
            c = sum(a * b for a, b in zip(w, ls))
            best = c if best is None or c < best else best
    return best


@pytest.mark.parametrize("seed", range(60))
def test_lengths_optimal_bruteforce(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 7))
    syms = rng.choice(256, size=k, replace=False)
    w = rng.integers(1, 12 if seed % 2 else 1000, size=k)
    h = np.zeros(256, dtype=np.uint64)
    h[syms] = w
    ln = oracle.code_lengths(h)
    cost = int(sum(int(h[v]) * int(ln[v]) for v in range(256)))
    assert cost == _brute_min_cost([int(x) for x in w])
    assert np.count_nonzero(ln) == k


def test_lengths_textbook_example():
    g = _golden("clrs_lengths.txt")
    h = _hist_of(_kv(g["count"], int))
    ln = oracle.code_lengths(h)
    for sym, l in _kv(g["len"], int).items():
        assert ln[ord(sym)] == l
    assert oracle.total_bits(h, ln) == int(g["cost"])


@pytest.mark.parametrize("m", [1, 2, 3, 8])
def test_lengths_uniform(m):
    h = np.zeros(256, dtype=np.uint64)
    h[: 1 << m] = 17
    ln = oracle.code_lengths(h)
    assert np.all(ln[: 1 << m] == m) and np.all(ln[1 << m:] == 0)


@pytest.mark.parametrize("lengths", [[1, 2, 3, 4, 4], [2, 2, 2, 3, 3], [1, 3, 3, 3, 4, 5, 5], [3] * 8])
def test_lengths_dyadic(lengths):
    """p_v = 2^-l_v with Kraft sum 1: the optimal lengths are l_v and L = H."""
    lmax = max(lengths)
    h = np.zeros(256, dtype=np.uint64)
    syms = np.arange(len(lengths)) * 7 + 3
    for s, l in zip(syms, lengths):
        h[s] = 1 << (lmax - l)
    ln = oracle.code_lengths(h)
    assert [int(ln[s]) for s in syms] == lengths
    n = int(h.sum())
    p = h[h > 0].astype(np.float64) / n
    ent = -(p * np.log2(p)).sum()
    assert abs(oracle.total_bits(h, ln) / n - ent) < 1e-12


@pytest.mark.parametrize("k", [2, 3, 6, 12, 20, 34])
def test_lengths_fibonacci(k):
    """Counts F_1..F_k give lengths (k-1, k-1, k-2, ..., 1): the deepest tree."""
    fib = [1, 1]
    while len(fib) < k:
        fib.append(fib[-1] + fib[-2])
    fib = fib[:k]
    h = np.zeros(256, dtype=np.uint64)
    h[:k] = fib
    ln = oracle.code_lengths(h)
    expect = [k - 1] + [k - i for i in range(1, k)]
    assert [int(x) for x in ln[:k]] == expect
    if k == 34:
        assert int(h.sum()) == 14_930_351 and ln.max() == 33


def test_lengths_special_cases():
    h = np.zeros(256, dtype=np.uint64)
    assert not oracle.code_lengths(h).any()
    h[65] = 10
    ln = oracle.code_lengths(h)
    assert ln[65] == 1 and np.count_nonzero(ln) == 1
    h[66] = 1
    ln = oracle.code_lengths(h)
    assert ln[65] == 1 and ln[66] == 1


def test_lengths_tie_rule():
    """{1,1,2,2}: with leaves first on equal weight all lengths are 2
    (internal-first would give 3,3,2,1: same cost, different code)."""
    h = np.zeros(256, dtype=np.uint64)
    h[[10, 11, 12, 13]] = [1, 1, 2, 2]
    assert [int(x) for x in oracle.code_lengths(h)[10:14]] == [2, 2, 2, 2]
    assert [int(x) for x in oracle.code_lengths(h, "twoqueue")[10:14]] == [2, 2, 2, 2]


@pytest.mark.parametrize("seed", range(200))
def test_lengths_heap_equals_twoqueue(seed):
    rng = np.random.default_rng(1000 + seed)
    k = int(rng.integers(1, 257))
    h = np.zeros(256, dtype=np.uint64)
    syms = rng.choice(256, size=k, replace=False)
    hi = [3, 10, 1000, 1 << 40][seed % 4]
    h[syms] = rng.integers(1, hi, size=k, dtype=np.uint64)
    assert np.array_equal(oracle.code_lengths(h), oracle.code_lengths(h, "twoqueue"))


def _kraft_exact(ln):
    ls = [int(x) for x in ln if x]
    lmax = max(ls)
    return sum(1 << (lmax - l) for l in ls), 1 << lmax


@pytest.mark.parametrize("name", ["zipf96_1MiB", "markov_45MiB"])
def test_lengths_kraft_and_entropy_on_workloads(name):
    a = datagen.workload(name, n=1 << 20)
    h = oracle.histogram(a)
    ln = oracle.code_lengths(h)
    s, full = _kraft_exact(ln)
    assert s == full
    n = a.size
    p = h[h > 0].astype(np.float64) / n
    ent = float(-(p * np.log2(p)).sum())
    lbar = oracle.total_bits(h, ln) / n
    assert ent - 1e-12 <= lbar < ent + 1.0
    assert oracle.total_bits(h, ln) == int(np.sum(ln[a].astype(np.uint64)))


@pytest.mark.parametrize("seed", range(40))
def test_lengths_kraft_random(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 257))
    h = np.zeros(256, dtype=np.uint64)
    h[rng.choice(256, size=k, replace=False)] = rng.integers(1, 10 ** int(rng.integers(1, 12)), size=k)
    ln = oracle.code_lengths(h)
    s, full = _kraft_exact(ln)
    assert s == full
    n = int(h.sum())
    p = h[h > 0].astype(np.float64) / n
    ent = float(-(p * np.log2(p)).sum())
    assert ent - 1e-9 <= oracle.total_bits(h, ln) / n < ent + 1.0


# ----------------------------------------------------------- canonical codes
def test_canonical_rfc1951_example():
    g = _golden("rfc1951_canonical.txt")
    ln = np.zeros(256, dtype=np.uint8)
    for sym, l in _kv(g["len"], int).items():
        ln[ord(sym)] = l
    code = oracle.canonical_codes(ln)
    for sym, bits in _kv(g["code"]).items():
        assert _bits(code[ord(sym)], ln[ord(sym)]) == bits


def test_canonical_hand_example():
    ln = np.zeros(256, dtype=np.uint8)
    ln[[ord("a"), ord("b"), ord("c"), ord("d")]] = [2, 1, 3, 3]
    code = oracle.canonical_codes(ln)
    got = {s: _bits(code[ord(s)], ln[ord(s)]) for s in "abcd"}
    assert got == {"a": "10", "b": "0", "c": "110", "d": "111"}


@pytest.mark.parametrize("seed", range(30))
def test_canonical_invariants(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 257))
    h = np.zeros(256, dtype=np.uint64)
    h[rng.choice(256, size=k, replace=False)] = rng.integers(1, 5000, size=k)
    ln = oracle.code_lengths(h)
    code = oracle.canonical_codes(ln)
    syms = [v for v in range(256) if ln[v]]
    strs = {v: _bits(code[v], ln[v]) for v in syms}
    # code fits its length
    assert all(int(code[v]) < (1 << int(ln[v])) for v in syms)
    # prefix-free: no code is a prefix of another
    ordered = sorted(strs.values())
    for x, y in zip(ordered, ordered[1:]):
        assert not y.startswith(x)
    # equal lengths: consecutive values in symbol order
    for l in set(int(ln[v]) for v in syms):
        same = [int(code[v]) for v in syms if ln[v] == l]
        assert same == list(range(same[0], same[0] + len(same)))
    # ordering by (length, symbol) equals numeric order of left-aligned codes
    lmax = int(ln.max())
    keyed = sorted(syms, key=lambda v: (int(ln[v]), v))
    left = [int(code[v]) << (lmax - int(ln[v])) for v in keyed]
    assert left == sorted(left)


# ------------------------------------------------------------------- encode
def _ref_encode_string(a, ln, code):
    """Independent bit layout: concatenate code strings, cut into MSB-first words."""
    s = "".join(_bits(code[x], ln[x]) for x in a)
    pad = (-len(s)) % 32
    s2 = s + "0" * pad
    words = [int(s2[i:i + 32], 2) for i in range(0, len(s2), 32)]
    return np.array(words, dtype=np.uint32), len(s)


def test_encode_golden_abracadabra():
    g = _golden("abracadabra.txt")
    a = np.frombuffer(g["input"].encode(), dtype=np.uint8)
    h = oracle.histogram(a)
    ln = oracle.code_lengths(h)
    code = oracle.canonical_codes(ln)
    for sym, l in _kv(g["len"], int).items():
        assert ln[ord(sym)] == l
    for sym, bits in _kv(g["code"]).items():
        assert _bits(code[ord(sym)], ln[ord(sym)]) == bits
    words, off = oracle.encode(a, ln, code, int(g["chunk"]))
    assert [int(w) for w in words] == [int(x, 16) for x in g["words"].split()]
    assert [int(o) for o in off] == [int(x) for x in g["chunk_off"].split()]
    assert int(off[-1]) == int(g["total_bits"])
    assert list(oracle.decode(words, off, a.size, int(g["chunk"]), ln)) == list(a)


@pytest.mark.parametrize("seed", range(25))
def test_encode_matches_string_reference(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3000))
    k = int(rng.integers(1, 40))
    syms = rng.choice(256, size=k, replace=False)
    a = rng.choice(syms, size=n, p=rng.dirichlet(np.ones(k) * 0.3)).astype(np.uint8)
    h = oracle.histogram(a)
    ln = oracle.code_lengths(h)
    code = oracle.canonical_codes(ln)
    words, off = oracle.encode(a, ln, code, 64)
    ref_words, t = _ref_encode_string(a, ln, code)
    assert np.array_equal(words, ref_words)
    assert int(off[-1]) == t == oracle.total_bits(h, ln)
    # chunk offsets are prefix sums of the per-byte lengths
    cum = np.concatenate([[0], np.cumsum(ln[a].astype(np.uint64))])
    idx = np.minimum(np.arange(0, (n + 63) // 64 + 1) * 64, n)
    assert np.array_equal(off, cum[idx].astype(np.uint64))


@pytest.mark.parametrize("chunks", [(1, 7, 1024), (16, 4096, 65536)])
def test_encode_independent_of_chunk(chunks):
    a = datagen.workload("markov_45MiB", n=200_000)
    h = oracle.histogram(a)
    ln = oracle.code_lengths(h)
    code = oracle.canonical_codes(ln)
    ref = None
    for c in chunks:
        words, off = oracle.encode(a, ln, code, c)
        assert off[0] == 0 and np.all(np.diff(off.astype(np.int64)) >= 0)
        assert int(off[-1]) == oracle.total_bits(h, ln)
        if ref is None:
            ref = words
        assert np.array_equal(words, ref)


def test_encode_empty_and_one_symbol():
    w, off = oracle.encode(np.zeros(0, np.uint8), np.zeros(256, np.uint8), np.zeros(256, np.uint64), 1024)
    assert w.size == 0 and list(off) == [0]
    a = np.full(100, 7, dtype=np.uint8)
    r = oracle.compress(a, 32)
    assert r["len"][7] == 1 and r["code"][7] == 0 and r["total_bits"] == 100
    assert np.all(r["words"] == 0) and r["words"].size == 4
    assert list(r["chunk_off"]) == [0, 32, 64, 96, 100]


def test_encode_rejects_symbol_without_code():
    ln = np.zeros(256, np.uint8)
    ln[1] = 1
    with pytest.raises(oracle.OracleError):
        oracle.encode(np.array([2], np.uint8), ln, np.zeros(256, np.uint64), 16)


# ------------------------------------------------------------------- decode
@pytest.mark.parametrize("name,n,chunk", [("zipf96_1MiB", 1 << 20, 65536), ("markov_45MiB", 300_001, 4096),
                                          ("zipf256_2GiB", 100_000, 1000)])
def test_roundtrip(name, n, chunk):
    a = datagen.workload(name, n=n)
    r = oracle.compress(a, chunk)
    out = oracle.decode(r["words"], r["chunk_off"], a.size, chunk, r["len"])
    assert np.array_equal(out, a)


def test_roundtrip_fibonacci_33_bits():
    fib = [1, 1]
    while len(fib) < 34:
        fib.append(fib[-1] + fib[-2])
    a = np.repeat(np.arange(34, dtype=np.uint8), fib)
    np.random.default_rng(0).shuffle(a)
    r = oracle.compress(a, 1 << 20)
    assert r["len"].max() == 33
    assert np.array_equal(oracle.decode(r["words"], r["chunk_off"], a.size, 1 << 20, r["len"]), a)


def test_decode_detects_corruption():
    a = datagen.workload("zipf96_1MiB", n=10_000)
    r = oracle.compress(a, 1024)
    bad = r["chunk_off"].copy()
    bad[3] += 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.decode(r["words"], bad, a.size, 1024, r["len"])
    assert e.value.code == oracle.CORRUPT
    with pytest.raises(oracle.OracleError):
        oracle.decode(r["words"][:-5], r["chunk_off"], a.size, 1024, r["len"])
    # a single-symbol code has only the code 0: a 1 bit is corrupt
    ln = np.zeros(256, np.uint8)
    ln[9] = 1
    with pytest.raises(oracle.OracleError):
        oracle.decode(np.array([0x80000000], np.uint32), np.array([0, 1], np.uint64), 1, 16, ln)
    assert list(oracle.decode(np.array([0], np.uint32), np.array([0, 1], np.uint64), 1, 16, ln)) == [9]


def test_sub_index_is_low_bits_of_fine_offsets():
    a = datagen.workload("markov_45MiB", n=50_000)
    r = oracle.compress(a, 4096, sub=256)
    _, fine = oracle.encode(a, r["len"], r["code"], 256)
    assert np.array_equal(r["sub_lo"], (fine & 0xFFFFFFFF).astype(np.uint32))
    assert r["sub_lo"].size == (a.size + 255) // 256 + 1


# ---------------------------------------------------------------- generators
def test_generators_deterministic_and_prefix_consistent():
    a = datagen.markov(3 << 20, 7)
    b = datagen.markov(3 << 20, 7)
    assert np.array_equal(a, b)
    c = datagen.markov((1 << 20) + 5, 7)
    assert np.array_equal(a[: c.size], c)
    z = datagen.zipf_iid(5000, 3, 1.1)
    assert set(np.unique(z)) <= set(datagen.A96.tolist())


def test_generator_shapes():
    a = datagen.workload("markov_45MiB", n=2 << 20)
    h = np.bincount(a, minlength=256)
    assert set(np.nonzero(h)[0]) <= set(datagen.A96.tolist())
    # lines: a newline within every ~70+4*15 bytes at most
    nl = np.nonzero(a == 10)[0]
    assert np.diff(nl).max() <= 70 + 15 * 8
    sizes = [datagen.file_params(5, i)[0] for i in range(200)]
    assert min(sizes) >= 4096 and max(sizes) <= 1 << 24
    mean_log = float(np.mean(np.log(sizes)))
    assert abs(mean_log - (math.log(4096) + math.log(1 << 24)) / 2) < 0.6
