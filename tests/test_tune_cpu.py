"""CPU checks of the launch-shape autotuner (paper_1010_0762_amd/tune.py):
candidate sets, the selection rule and the JSON cache, with a synthetic
timing function in place of the GPU."""
import json

from paper_1010_0762_amd import tune
from paper_1010_0762_amd import workloads as wl


def test_candidates_cover_the_rows():
    # 64^3: at least 32 blocks (8 rows per thread), at most 256 with rows
    c = tune.candidates(64 ** 3)
    blocks = sorted({b for b, _ in c})
    assert blocks == [0, 64, 128, 256]
    assert {ch for _, ch in c} == {4, 8, 16}
    # 128^3 needs at least 256 blocks
    assert sorted({b for b, _ in tune.candidates(128 ** 3)}) == [0, 256, 512, 1024]
    # tiny: the automatic grid only
    assert sorted({b for b, _ in tune.candidates(1000)}) == [0]


def test_pick_and_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    A = wl.convdiff(16, 3, [20.0, 10.0, 5.0])
    calls = []

    def fake(blocks, chunk):
        calls.append((blocks, chunk))
        return 1e-5 * (1 + abs(chunk - 8) / 8)      # chunk 8 best, blocks indifferent

    cands = [(0, 4), (0, 8), (0, 16)]
    e = tune.autotune(A, k=10, s=20, cache=path, cands=cands, repeats=2, measure=fake)
    assert (e["blocks"], e["chunk"]) == (0, 8) and not e["cached"]
    assert len(calls) == 6
    data = json.load(open(path))
    assert len(data) == 1 and list(data.values())[0]["chunk"] == 8
    # a second call reads the cache and times nothing
    e2 = tune.autotune(A, k=10, s=20, cache=path, cands=cands, measure=fake)
    assert e2["cached"] and len(calls) == 6
    assert tune.lookup(A, k=10, s=20, cache=path, device="cpu")["chunk"] == 8
    # another shape is another entry
    tune.autotune(A, k=20, s=20, cache=path, cands=cands, measure=fake)
    assert len(json.load(open(path))) == 2


def test_pick_prefers_automatic_on_ties():
    t = {(0, 8): 1.0, (256, 8): 1.0, (128, 16): 1.0}
    assert tune.pick(t) == (0, 8)
    t = {(256, 8): 1.0, (128, 16): 1.0}
    assert tune.pick(t) == (128, 16)
