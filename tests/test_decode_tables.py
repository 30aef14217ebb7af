"""Host checks of the index arithmetic the longer-code decoder relies on,
against the oracle's canonical codes (Section III.A's tree, read as a
canonical code with shorter codes numerically first): the codes of at most
12 bits cover exactly the first P 12-bit prefixes, every longer code starts
with one of the last 4096 - P, and the second table -- entry
(maxLen-bit peek) - P * 2^(maxLen - 12), (4096 - P) * 2^(maxLen - 12) entries
-- holds each longer code on exactly the entries its bits select.  The
kernels are not run here; this pins the layout they build."""
import numpy as np
import pytest

import datagen
import oracle

WIDE = 12


def _tables(lengths, codes):
    ln = np.asarray(lengths, dtype=np.int64)
    cd = np.asarray(codes, dtype=np.uint64)
    L = int(ln.max())
    cnt = np.bincount(ln[ln > 0], minlength=64)
    P = sum(int(cnt[l]) << (WIDE - l) for l in range(1, WIDE + 1))
    return ln, cd, L, P


def _cases():
    out = []
    for s, n in [(1.4, 1 << 20), (1.6, 1 << 20), (1.8, 1 << 20), (2.0, 1 << 20), (2.2, 1 << 20), (1.5, 300_001), (1.7, 300_001)]:
        a = datagen.zipf_iid(n, 3, s, datagen.A256)
        out.append((f"zipf{s}", np.bincount(a, minlength=256).astype(np.uint64)))
    # dyadic counts: lengths 1, 2, ..., L, L
    for L in (13, 16, 20):
        h = np.zeros(256, np.uint64)
        for i in range(L):
            h[i * 7 + 3] = 1 << (L - 1 - i)
        h[L * 7 + 3] = 1
        out.append((f"dyadic{L}", h))
    # Fibonacci counts: a chain of ever longer codes
    h = np.zeros(256, np.uint64)
    f0, f1 = 1, 1
    for i in range(24):
        h[i] = f0
        f0, f1 = f1, f0 + f1
    out.append(("fib24", h))
    return out


@pytest.mark.parametrize("name,hist", _cases(), ids=[c[0] for c in _cases()])
def test_second_table_layout(name, hist):
    ln = oracle.code_lengths(hist)
    cd = oracle.canonical_codes(ln)
    ln, cd, L, P = _tables(ln, cd)
    assert L > WIDE
    # every 12-bit prefix below P starts a code of at most 12 bits, none at or above it
    short = np.zeros(1 << WIDE, bool)
    for v in np.nonzero((ln > 0) & (ln <= WIDE))[0]:
        l = int(ln[v])
        p0 = int(cd[v]) << (WIDE - l)
        assert not short[p0:p0 + (1 << (WIDE - l))].any()
        short[p0:p0 + (1 << (WIDE - l))] = True
    assert short[:P].all() and not short[P:].any()
    # the longer codes fill the second table exactly once each
    extra = L - WIDE
    n2 = ((1 << WIDE) - P) << extra
    base = P << extra
    owner = np.full(n2, -1, np.int64)
    for v in np.nonzero(ln > WIDE)[0]:
        l = int(ln[v])
        assert (int(cd[v]) >> (l - WIDE)) >= P  # starts with one of the last prefixes
        e0 = (int(cd[v]) << (L - l)) - base
        e1 = e0 + (1 << (L - l))
        assert 0 <= e0 and e1 <= n2
        assert (owner[e0:e1] == -1).all()
        owner[e0:e1] = v
    # a complete code leaves no entry empty; the decoder's index never leaves the table
    assert (owner >= 0).all()
    for top in np.random.default_rng(0).integers(0, 1 << 32, 2000, dtype=np.uint64):
        idx = int(top) >> (32 - WIDE)
        if idx >= P and L <= 32:
            i2 = (int(top) >> (32 - L)) - base
            assert 0 <= i2 < n2
            v = owner[i2]
            l = int(ln[v])
            assert int(top) >> (32 - l) == int(cd[v])  # the entry's code is the one the bits start with
