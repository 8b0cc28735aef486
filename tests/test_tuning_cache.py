"""The autotuner's JSON cache (host code): entries per (arch, D, Q, R, bin), merged on
store, written atomically, only for the bins that were timed."""

import json

from paper_1411_4283_amd import api
from paper_1411_4283_amd._lib import Tuning


def _tuning(vals):
    t = Tuning()
    for b, (x, p, s) in enumerate(vals):
        t.xcd_chunks[b], t.blocks_per_xcd[b], t.split[b] = x, p, s
    return t


def test_store_keeps_timed_bins_and_merges(tmp_path):
    path = str(tmp_path / "t.json")
    t1 = _tuning([(1, 0, 0), (8, 0, 1), (8, 128, 2), (1, 0, 3)] + [(1, 0, 0)] * 4)
    api._cache_store(path, "gfx950/D3/Q4/R3", t1, [-1.0, 0.5, 1.5, 2.5, -1.0, -1.0, -1.0, -1.0])
    e = json.load(open(path))
    assert sorted(e) == ["gfx950/D3/Q4/R3/bin1", "gfx950/D3/Q4/R3/bin2", "gfx950/D3/Q4/R3/bin3"]
    assert e["gfx950/D3/Q4/R3/bin2"] == {"xcd_chunks": 8, "blocks_per_xcd": 128, "split": 2, "best_ms": 1.5}
    # another shape adds its own keys; a retune of the same bin replaces its entry
    t2 = _tuning([(8, 0, 1)] * 8)
    api._cache_store(path, "gfx950/D2/Q4/R3", t2, [0.1] + [-1.0] * 7)
    api._cache_store(path, "gfx950/D3/Q4/R3", t2, [-1.0, -1.0, 0.7] + [-1.0] * 5)
    e = api._cache_load(path)
    assert "gfx950/D2/Q4/R3/bin0" in e and len(e) == 4
    assert e["gfx950/D3/Q4/R3/bin2"]["split"] == 1 and e["gfx950/D3/Q4/R3/bin1"]["split"] == 1
    assert not list(tmp_path.glob("*.tmp*"))


def test_missing_file_is_an_empty_cache(tmp_path):
    assert api._cache_load(str(tmp_path / "none.json")) == {}
