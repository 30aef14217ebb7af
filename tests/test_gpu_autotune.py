"""GPU run of the autotuner on a small input with a reduced search space:
it returns a complete setting, caches it, and the tuned launch parameters
give the same bits as the defaults (parameters only change how the work is
split)."""
import sys

import numpy as np
import pytest

import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_tune_small_space_and_cache(tmp_path):
    import paper_2306_11070_amd as P
    from paper_2306_11070_amd import autotune as A
    P.load()
    _say("autotune 4 MiB markov, reduced space")
    a = datagen.markov(4 << 20, 91)
    x = torch.from_numpy(a).cuda()
    space = {"hist_depth": [4, 16], "hist_blocks_per_cu": [2, 4], "enc_blocks_per_cu": [2, 3],
             "sub_size": [0, 128], "dec_block": [256]}
    cache = A.Cache(str(tmp_path / "tune.json"))
    r = A.tune(x, space=space, reps=2, cache=cache)
    for k in ("hist_depth", "hist_blocks", "enc_blocks_per_cu", "sub_size", "dec_block", "chunk_size"):
        assert k in r, k
    assert r["hist_depth"] in (4, 16) and r["sub_size"] in (0, 128) and r["enc_blocks_per_cu"] in (2, 3)
    assert r["chunk_size"] in A.DEFAULT_SPACE["chunk_size"]
    assert A.Cache(str(tmp_path / "tune.json")).get(r["key"]) is not None
    again = A.tune(x, space=space, reps=2, cache=cache)  # from the cache
    assert again == r
    # tuned launch parameters give the same stream as the defaults
    tuned = P.Codec(0, A.params_of(r))
    base = P.Codec(0)
    c1 = tuned.compress(x, r["chunk_size"], r["sub_size"])
    c2 = base.compress(x, r["chunk_size"], r["sub_size"])
    torch.cuda.synchronize()
    nw = (int(c2["chunk_off"][-1].item()) + 31) // 32
    assert torch.equal(c1["words"][:nw], c2["words"][:nw]) and torch.equal(c1["chunk_off"], c2["chunk_off"])
    out = tuned.decompress(c1)
    assert torch.equal(out, x)
    tuned.close()
    base.close()
