"""CPU tests of the autotuner's host logic (no GPU): the cache, the workload
key, the index budget and the selection rules."""
import json

from paper_2306_11070_amd import autotune as A


def test_index_bytes_matches_layout():
    # 8 bytes per chunk entry (nchunks + 1), 4 per sub-block entry (nsub + 1)
    assert A.index_bytes(0, 1024, 0) == 8
    assert A.index_bytes(1, 1024, 0) == 16
    assert A.index_bytes(4096, 1024, 0) == 8 * 5
    assert A.index_bytes(4096, 1024, 64) == 8 * 5 + 4 * 65
    assert A.index_bytes(4097, 1024, 64) == 8 * 6 + 4 * 66


def test_pick_min_first_on_ties():
    assert A.pick_min({"a": 3.0, "b": 1.0, "c": 1.0}) == "b"
    assert A.pick_min({(1, 2): 0.5}) == (1, 2)
    assert A.pick_min({}) is None


def test_choose_chunk_respects_budget():
    n = 1 << 30
    payload = int(n * 6.65 / 8)
    chunks = A.DEFAULT_SPACE["chunk_size"]
    c = A.choose_chunk(n, payload, 256, chunks, 0.03)
    assert A.index_bytes(n, c, 256) <= 0.03 * payload
    smaller = [x for x in chunks if x < c]
    assert all(A.index_bytes(n, x, 256) > 0.03 * payload for x in smaller)
    # impossible budget: the largest candidate
    assert A.choose_chunk(n, payload, 16, chunks, 1e-9) == max(chunks)
    # never below the sub-block size or 1 KiB
    assert A.choose_chunk(1 << 20, 1 << 20, 0, [512, 1024, 2048], 1.0) == 1024


def test_workload_key_buckets():
    k1 = A.workload_key("MI355X", 256, 47_185_920, 6.65)
    k2 = A.workload_key("MI355X", 256, 40_000_000, 6.9)
    k3 = A.workload_key("MI355X", 256, 1 << 31, 6.65)
    assert k1 == k2 and k1 != k3
    assert "cu256" in k1 and "bpb7" in k1


def test_cache_roundtrip(tmp_path):
    p = tmp_path / "sub" / "tune.json"
    c = A.Cache(str(p))
    assert c.get("k") is None
    c.put("k", {"hist_depth": 8, "x": 1.5})
    assert json.loads(p.read_text())["k"]["hist_depth"] == 8
    c2 = A.Cache(str(p))
    assert c2.get("k") == {"hist_depth": 8, "x": 1.5}
    p.write_text("{not json")
    assert A.Cache(str(p)).get("k") is None  # a damaged cache is ignored


def test_params_of():
    t = {"hist_blocks": 512, "hist_depth": 16, "dec_block": 256, "enc_blocks_per_cu": 3, "sub_size": 64}
    assert A.params_of(t) == {"hist_blocks": 512, "hist_depth": 16, "dec_block": 256, "enc_blocks_per_cu": 3}
